// C ABI of libcg (include/cg.h): contexts, scratch sizing, host-side
// argument checks and the five steps of Algorithm 2.  No exception leaves
// this file; every entry point returns a status code.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "cg_internal.h"

namespace cg {

static thread_local char g_err[512] = "";

int set_error(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return CG_OK;
  return set_error(CG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout(int64_t n, int64_t m, int64_t P) {
  (void)m;
  Layout L{};
  const int64_t nn = n > 0 ? n : 1;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t here = at;
    at += align_up(bytes);
    return here;
  };
  L.scan_status = take(sizeof(unsigned long long) * (size_t)(scan_blocks(nn + 1) + 1));
  L.tmp = take(8 * (size_t)nn);
  L.lidx = take(4 * (size_t)nn);
  L.fill = take(4 * (size_t)nn);
  L.piece_off = take(8 * (size_t)nn);
  L.piece_len = take(4 * (size_t)nn);
  L.lay_contig = take(4 * (size_t)nn);
  L.keys = take(8 * (size_t)(2 * nn + 2));
  L.bins = take(8 * (size_t)(2 * (P > 0 ? P : 1)));
  L.aux = take(4 * (size_t)nn);
  L.walk = take(4 * 16 * (size_t)nn);
  L.estart = take(4 * (size_t)nn);
  L.memb = take(4 * (size_t)nn);
  L.piece_src = take(8 * (size_t)nn);
  L.comp_w = take(8 * (size_t)nn);
  L.bin_reads = take(8 * (size_t)(P > 0 ? P : 1));
  L.total = at;
  return L;
}

bool carve(cg_ctx *ctx, int64_t n, int64_t m, int64_t P, Scratch *s) {
  Layout L = layout(n, m, P);
  if (L.total > ctx->scratch_bytes) return false;
  char *b = ctx->scratch;
  s->scan_status = (unsigned long long *)(b + L.scan_status);
  s->tmp = (int32_t *)(b + L.tmp);
  s->lidx = (int32_t *)(b + L.lidx);
  s->fill = (uint32_t *)(b + L.fill);
  s->piece_off = (uint64_t *)(b + L.piece_off);
  s->piece_len = (uint32_t *)(b + L.piece_len);
  s->lay_contig = (int32_t *)(b + L.lay_contig);
  s->keys = (uint64_t *)(b + L.keys);
  s->bins = (uint64_t *)(b + L.bins);
  s->aux = (int32_t *)(b + L.aux);
  s->walk = (int32_t *)(b + L.walk);
  s->estart = (int32_t *)(b + L.estart);
  s->memb = (int32_t *)(b + L.memb);
  s->piece_src = (uint64_t *)(b + L.piece_src);
  s->comp_w = (uint64_t *)(b + L.comp_w);
  s->bin_reads = (uint64_t *)(b + L.bin_reads);
  return true;
}

int prof_begin(cg_ctx *ctx, hipStream_t st, const char *name) {
  if (!ctx || !ctx->prof) return -1;
  if (ctx->prof_used >= ctx->prof_cap) {
    ++ctx->prof_dropped;
    return -1;
  }
  const int slot = ctx->prof_used++;
  ctx->prof[slot].name = name;
  (void)hipEventRecord(ctx->prof[slot].a, st);
  return slot;
}

void prof_end(cg_ctx *ctx, hipStream_t st, int slot) {
  if (slot >= 0) (void)hipEventRecord(ctx->prof[slot].b, st);
}

static void prof_free(cg_ctx *ctx) {
  if (!ctx->prof) return;
  for (int i = 0; i < ctx->prof_cap; ++i) {
    (void)hipEventDestroy(ctx->prof[i].a);
    (void)hipEventDestroy(ctx->prof[i].b);
  }
  delete[] ctx->prof;
  ctx->prof = nullptr;
  ctx->prof_cap = ctx->prof_used = 0;
  ctx->prof_dropped = 0;
}

}  // namespace cg

using namespace cg;

int cg::check_graph(const cg_graph *g, bool need_seq) {
  if (!g) return set_error(CG_EINVAL, "graph is NULL");
  if (g->n < 0 || g->n >= (1 << 30)) return set_error(CG_EINVAL, "n=%d outside [0, 2^30)", g->n);
  if (g->m < 0) return set_error(CG_EINVAL, "m=%d is negative", g->m);
  if (!g->row_ptr) return set_error(CG_EINVAL, "row_ptr is NULL");
  if (g->m > 0 && (!g->col || !g->ovl || !g->strand))
    return set_error(CG_EINVAL, "col/ovl/strand is NULL");
  if (need_seq && g->n > 0 && (!g->read_len || !g->read_off || !g->seq))
    return set_error(CG_EINVAL, "read_len/read_off/seq is NULL");
  if ((g->pre == nullptr) != (g->post == nullptr))
    return set_error(CG_EINVAL, "pre and post must both be given or both be NULL");
  return CG_OK;
}

int cg::check_P(int32_t P) {
  if (P < 1 || P > 65536) return set_error(CG_EINVAL, "P=%d outside [1, 65536]", P);
  return CG_OK;
}

int cg::check_parts(const cg_parts *p) {
  if (!p || !p->comp_label || !p->comp_size || !p->comp_kind || !p->comp_bin || !p->comp_rank ||
      !p->comp_start || !p->bin_load || !p->label_comp || !p->d_n_comp)
    return set_error(CG_EINVAL, "cg_parts has a NULL member");
  return CG_OK;
}

int cg::check_local(const cg_local *l) {
  if (!l || !l->perm || !l->bin_vptr || !l->loc_row_ptr || !l->loc_col || !l->loc_eid ||
      !l->d_sizes)
    return set_error(CG_EINVAL, "cg_local has a NULL member");
  return CG_OK;
}

int cg::check_contigs(const cg_contigs *c) {
  if (!c || !c->label || !c->bin || !c->start || !c->n_reads || !c->len || !c->base_off ||
      !c->cflags || !c->layout_off || !c->layout_vid || !c->layout_rev || !c->d_total_words ||
      (c->cap_words > 0 && !c->bases))
    return set_error(CG_EINVAL, "cg_contigs has a NULL member");
  return CG_OK;
}

static int check_ctx(cg_ctx *ctx, const cg_graph *g, int32_t P, Scratch *s) {
  if (!ctx) return set_error(CG_EINVAL, "context is NULL");
  if (!carve(ctx, g->n, g->m, P, s))
    return set_error(CG_ENOMEM, "context scratch of %zu bytes is below the %zu bytes needed",
                     ctx->scratch_bytes, layout(g->n, g->m, P).total);
  return CG_OK;
}

extern "C" {

const char *cg_last_error(void) { return g_err; }

int cg_footprint(int32_t n, int32_t m, uint64_t seq_words, int32_t P, int32_t coords,
                 cg_sizes *out) {
  if (!out || n < 0 || m < 0 || P < 1 || P > 65536 || seq_words >= (1ull << 62))
    return set_error(CG_EINVAL, "bad footprint arguments (n=%d m=%d P=%d)", n, m, P);
  const uint64_t N = (uint64_t)n, M = (uint64_t)m, Pb = (uint64_t)P;
  out->scratch = (uint64_t)layout(n, m, P).total;
  // row_ptr, col, ovl, strand, read_len, read_off, seq (+ pre, post)
  out->graph = 4 * (N + 1) + M * (4 + 4 + 1) + N * (4 + 8) + 4 * seq_words +
               (coords ? 8 * M : 0);
  // per read: flags 1, label 4; cg_parts: comp_label, comp_size 8, comp_kind 1,
  // comp_bin, comp_rank, comp_start 12, label_comp 4; cg_local: perm 4,
  // loc_row_ptr 4 (+4 once), loc_col, loc_eid 16; cg_contigs: label, bin,
  // start, n_reads 16, len, base_off 16, cflags, layout_off 8, layout_vid 4,
  // layout_rev 1 -- 99 bytes; then d_counts 8, bin_load 8P, d_n_comp 4,
  // bin_vptr 4(P+1), d_sizes 8, bases 4 cap_words, d_total_words 8
  out->outputs = 99 * N + 4 + 8 + 8 * Pb + 4 + 4 * (Pb + 1) + 8 + 4 * seq_words + 8;
  return CG_OK;
}

int cg_job_outputs(int32_t n, int32_t P, uint64_t cap_words, void *base, uint64_t *bytes,
                   cg_job *job) {
  if (!bytes || n < 0 || P < 1 || P > 65536 || cap_words >= (1ull << 62) ||
      (base && (!job || ((uintptr_t)base & 255))))
    return set_error(CG_EINVAL, "bad arguments (n=%d P=%d, base 256-byte aligned with a job)",
                     n, P);
  const uint64_t k = n > 0 ? (uint64_t)n : 1, Pb = (uint64_t)P;
  const uint64_t words = cap_words > 0 ? cap_words : 1;
  char *b = (char *)base;
  uint64_t at = 0;
  // each buffer at the next 256-byte boundary
  auto take = [&](uint64_t size) -> void * {
    void *p = b ? (void *)(b + at) : nullptr;
    at += (size + 255) & ~(uint64_t)255;
    return p;
  };
  cg_job j{};
  j.flags = (uint8_t *)take(k);
  j.d_counts = (int32_t *)take(8);
  j.label = (int32_t *)take(4 * k);
  j.parts.comp_label = (int32_t *)take(4 * k);
  j.parts.comp_size = (int32_t *)take(4 * k);
  j.parts.comp_kind = (uint8_t *)take(k);
  j.parts.comp_bin = (int32_t *)take(4 * k);
  j.parts.comp_rank = (int32_t *)take(4 * k);
  j.parts.comp_start = (int32_t *)take(4 * k);
  j.parts.bin_load = (uint64_t *)take(8 * Pb);
  j.parts.label_comp = (int32_t *)take(4 * k);
  j.parts.d_n_comp = (int32_t *)take(4);
  j.local.perm = (int32_t *)take(4 * k);
  j.local.bin_vptr = (int32_t *)take(4 * (Pb + 1));
  j.local.loc_row_ptr = (int32_t *)take(4 * (k + 1));
  j.local.loc_col = (int32_t *)take(8 * k);
  j.local.loc_eid = (int32_t *)take(8 * k);
  j.local.d_sizes = (int32_t *)take(8);
  j.contigs.label = (int32_t *)take(4 * k);
  j.contigs.bin = (int32_t *)take(4 * k);
  j.contigs.start = (int32_t *)take(4 * k);
  j.contigs.n_reads = (int32_t *)take(4 * k);
  j.contigs.len = (uint64_t *)take(8 * k);
  j.contigs.base_off = (uint64_t *)take(8 * k);
  j.contigs.cflags = (uint32_t *)take(4 * k);
  j.contigs.layout_off = (int32_t *)take(4 * k);
  j.contigs.layout_vid = (int32_t *)take(4 * k);
  j.contigs.layout_rev = (uint8_t *)take(k);
  j.contigs.bases = (uint32_t *)take(4 * words);
  j.contigs.cap_words = cap_words;
  j.contigs.d_total_words = (uint64_t *)take(8);
  *bytes = at;
  if (b) {
    job->flags = j.flags;
    job->d_counts = j.d_counts;
    job->label = j.label;
    job->parts = j.parts;
    job->local = j.local;
    job->contigs = j.contigs;
  }
  return CG_OK;
}

int cg_ctx_create(int device, size_t scratch_bytes, cg_ctx **out) {
  if (!out) return set_error(CG_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  int rc = hip_check(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (rc) return rc;
  if (device < 0 || device >= ndev) return set_error(CG_EINVAL, "device %d of %d", device, ndev);
  int prev = 0;
  (void)hipGetDevice(&prev);
  if ((rc = hip_check(hipSetDevice(device), "hipSetDevice"))) return rc;
  cg_ctx *c = new (std::nothrow) cg_ctx();
  if (!c) return set_error(CG_EINVAL, "out of host memory");
  c->device = device;
  c->scratch_bytes = scratch_bytes;
  c->scratch = nullptr;
  c->fixed = nullptr;
  c->prof = nullptr;
  c->prof_cap = c->prof_used = 0;
  c->prof_dropped = 0;
  rc = hip_check(hipMalloc((void **)&c->fixed, sizeof(Fixed)), "hipMalloc(fixed)");
  if (!rc) rc = hip_check(hipMemset(c->fixed, 0, sizeof(Fixed)), "hipMemset(fixed)");
  if (!rc && scratch_bytes)
    rc = hip_check(hipMalloc((void **)&c->scratch, scratch_bytes), "hipMalloc(scratch)");
  if (!rc && scratch_bytes)
    rc = hip_check(hipMemset(c->scratch, 0, scratch_bytes), "hipMemset(scratch)");
  if (!rc) rc = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
  (void)hipSetDevice(prev);
  if (rc) {
    if (c->scratch) (void)hipFree(c->scratch);
    if (c->fixed) (void)hipFree(c->fixed);
    delete c;
    return rc;
  }
  *out = c;
  return CG_OK;
}

int cg_ctx_destroy(cg_ctx *ctx) {
  if (!ctx) return CG_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  int rc = CG_OK;
  prof_free(ctx);
  if (ctx->scratch) rc = hip_check(hipFree(ctx->scratch), "hipFree(scratch)");
  if (ctx->fixed && !rc) rc = hip_check(hipFree(ctx->fixed), "hipFree(fixed)");
  (void)hipSetDevice(prev);
  delete ctx;
  return rc;
}

int cg_ctx_status(cg_ctx *ctx, void *stream, uint32_t *status, int clear) {
  if (!ctx || !status) return set_error(CG_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  int rc = hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (rc) return rc;
  rc = hip_check(hipMemcpy(status, &ctx->fixed->status, sizeof(uint32_t), hipMemcpyDeviceToHost),
                 "hipMemcpy(status)");
  if (rc) return rc;
  if (clear)
    rc = hip_check(hipMemset(&ctx->fixed->status, 0, sizeof(uint32_t)), "hipMemset(status)");
  return rc;
}

int cg_ctx_profile(cg_ctx *ctx, int32_t max_launches) {
  if (!ctx || max_launches < 0) return set_error(CG_EINVAL, "bad profile arguments");
  prof_free(ctx);
  if (max_launches == 0) return CG_OK;
  ctx->prof = new (std::nothrow) ProfEntry[max_launches];
  if (!ctx->prof) return set_error(CG_EINVAL, "out of host memory");
  for (int i = 0; i < max_launches; ++i) {
    ctx->prof[i].name = nullptr;
    int rc = hip_check(hipEventCreate(&ctx->prof[i].a), "hipEventCreate");
    if (!rc) rc = hip_check(hipEventCreate(&ctx->prof[i].b), "hipEventCreate");
    if (rc) {
      ctx->prof_cap = i;
      prof_free(ctx);
      return rc;
    }
    ctx->prof_cap = i + 1;
  }
  ctx->prof_used = 0;
  return CG_OK;
}

int cg_ctx_profile_read(cg_ctx *ctx, int32_t cap, const char **names, int64_t *launches,
                        double *ms, int32_t *n_kernels, int64_t *dropped) {
  if (!ctx || !n_kernels || cap < 0 || (cap > 0 && (!names || !launches || !ms)))
    return set_error(CG_EINVAL, "bad profile_read arguments");
  int k = 0;
  for (int i = 0; i < ctx->prof_used; ++i) {
    int rc = hip_check(hipEventSynchronize(ctx->prof[i].b), "hipEventSynchronize");
    if (rc) return rc;
    float t = 0.f;
    rc = hip_check(hipEventElapsedTime(&t, ctx->prof[i].a, ctx->prof[i].b), "hipEventElapsedTime");
    if (rc) return rc;
    int j = 0;
    while (j < k && strcmp(names[j], ctx->prof[i].name) != 0) ++j;
    if (j == k) {
      if (k == cap) return set_error(CG_ECAPACITY, "more than %d kernel names", cap);
      names[k] = ctx->prof[i].name;
      launches[k] = 0;
      ms[k] = 0.0;
      ++k;
    }
    launches[j] += 1;
    ms[j] += t;
  }
  *n_kernels = k;
  if (dropped) *dropped = ctx->prof_dropped;
  ctx->prof_used = 0;
  ctx->prof_dropped = 0;
  return CG_OK;
}

int cg_validate(cg_ctx *ctx, const cg_graph *g, int64_t *d_bad, void *stream) {
  int rc = check_graph(g, true);
  if (rc) return rc;
  if (!ctx || !d_bad) return set_error(CG_EINVAL, "NULL argument");
  return launch_validate(ctx, *g, d_bad, (hipStream_t)stream);
}

int cg_reduce(cg_ctx *ctx, const cg_graph *r, uint32_t fuzz, uint8_t *contained, uint8_t *kept,
              int32_t *s_row_ptr, int32_t *s_col, uint32_t *s_ovl, uint8_t *s_strand,
              int32_t *d_m, void *stream) {
  int rc = check_graph(r, false);
  if (rc) return rc;
  if (!s_row_ptr || !d_m || (r->n > 0 && (!contained || !r->read_len)) ||
      (r->m > 0 && (!kept || !s_col || !s_ovl || !s_strand)))
    return set_error(CG_EINVAL, "NULL argument");
  Scratch s;
  if ((rc = check_ctx(ctx, r, 1, &s))) return rc;
  return launch_reduce(ctx, *r, s, fuzz, contained, kept, s_row_ptr, s_col, s_ovl, s_strand, d_m,
                       (hipStream_t)stream);
}

int cg_mask_branches(cg_ctx *ctx, const cg_graph *g, uint8_t *flags, int32_t *d_counts,
                     void *stream) {
  int rc = check_graph(g, false);
  if (rc) return rc;
  if (!ctx || !d_counts || (g->n > 0 && !flags)) return set_error(CG_EINVAL, "NULL argument");
  return launch_mask(ctx, *g, flags, d_counts, (hipStream_t)stream);
}

int cg_components(cg_ctx *ctx, const cg_graph *g, const uint8_t *flags, int32_t *label,
                  void *stream) {
  int rc = check_graph(g, false);
  if (rc) return rc;
  if (!ctx || (g->n > 0 && (!flags || !label))) return set_error(CG_EINVAL, "NULL argument");
  return launch_components(ctx, *g, flags, label, (hipStream_t)stream);
}

int cg_partition(cg_ctx *ctx, const cg_graph *g, const uint8_t *flags, const int32_t *label,
                 int32_t P, int32_t min_reads, int32_t weight, const cg_parts *out,
                 void *stream) {
  int rc = check_graph(g, false);
  if (rc || (rc = check_P(P)) || (rc = check_parts(out))) return rc;
  if (g->n > 0 && (!flags || !label)) return set_error(CG_EINVAL, "NULL argument");
  if (weight != CG_WEIGHT_READS && weight != CG_WEIGHT_BASES)
    return set_error(CG_EINVAL, "weight=%d is neither CG_WEIGHT_READS nor CG_WEIGHT_BASES", weight);
  if (weight == CG_WEIGHT_BASES && g->n > 0 && !g->read_len)
    return set_error(CG_EINVAL, "bases weights need read_len");
  Scratch s;
  if ((rc = check_ctx(ctx, g, P, &s))) return rc;
  return launch_partition(ctx, *g, s, flags, label, P, min_reads, weight, *out,
                          (hipStream_t)stream);
}

int cg_induce(cg_ctx *ctx, const cg_graph *g, const uint8_t *flags, const int32_t *label,
              const cg_parts *parts, int32_t P, const cg_local *out, void *stream) {
  int rc = check_graph(g, false);
  if (rc || (rc = check_P(P)) || (rc = check_parts(parts))) return rc;
  if ((rc = check_local(out))) return rc;
  if (g->n > 0 && (!flags || !label)) return set_error(CG_EINVAL, "NULL argument");
  Scratch s;
  if ((rc = check_ctx(ctx, g, P, &s))) return rc;
  return launch_induce(ctx, *g, s, flags, label, *parts, P, *out, (hipStream_t)stream);
}

int cg_assemble(cg_ctx *ctx, const cg_graph *g, const cg_parts *parts, const cg_local *local,
                int32_t P, const cg_contigs *out, void *stream) {
  int rc = check_graph(g, true);
  if (rc || (rc = check_P(P)) || (rc = check_parts(parts))) return rc;
  if (!local || !local->perm || !local->bin_vptr || !local->loc_row_ptr || !local->loc_col ||
      !local->loc_eid)
    return set_error(CG_EINVAL, "cg_local has a NULL member");
  if ((rc = check_contigs(out))) return rc;
  Scratch s;
  if ((rc = check_ctx(ctx, g, P, &s))) return rc;
  return launch_assemble(ctx, *g, s, *parts, *local, P, *out, (hipStream_t)stream);
}

}  // extern "C"
