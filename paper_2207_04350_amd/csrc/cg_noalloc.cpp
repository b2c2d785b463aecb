// Allocation-free form of ContigGeneration (Algorithm 2) on one graph: the
// five steps with the same launchers and kernels as the context calls, their
// scratch taken from a static device array instead of a context.
//
// The array is one per GPU: the loader places a copy of every __device__
// variable on each device the code object is loaded on.  Its host-side name
// is only a stand-in for the device copy, so its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is ever handed to kernels.
#include <mutex>

#include "cg_internal.h"

namespace cg {

// [Fixed | context scratch of CG_NOALLOC_SCRATCH_BYTES]
constexpr size_t kFixedBytes = (sizeof(Fixed) + 255) & ~(size_t)255;
constexpr size_t kStaticBytes = kFixedBytes + (size_t)CG_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_mu;
static char *g_ptr[kMaxDevices];  // device address of `scratch` per device (null: not looked up)

// The device address of this device's copy of `scratch`, looked up on the
// first call that runs on the device.
static int scratch_on(int dev, char **out) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(CG_EUNSUPPORTED, "device %d", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    int rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    if (rc) return rc;
    g_ptr[dev] = (char *)p;
  }
  *out = g_ptr[dev];
  return CG_OK;
}

// What must start at zero: the counters the kernels count on (they reset
// them themselves after use, but a call must not depend on how the previous
// one ended), the status word, and the look-back status of this call's scans.
__global__ void k_noalloc_reset(Fixed *fx, unsigned long long *scan_status, int n_status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    fx->mask_ticket = 0;
    fx->status = 0;
    fx->scan_ticket = 0;
    fx->scan_done = 0;
  }
  for (int i = t; i < n_status; i += gridDim.x * blockDim.x) scan_status[i] = 0;
}

__global__ void k_noalloc_status(const Fixed *fx, uint32_t *d_status) { *d_status = fx->status; }

}  // namespace cg

using namespace cg;

extern "C" int cg_contig_generation_noalloc(const cg_graph *g, int32_t P, int32_t min_reads,
                                            int32_t weight, uint8_t *flags, int32_t *d_counts,
                                            int32_t *label, const cg_parts *parts,
                                            const cg_local *local, const cg_contigs *contigs,
                                            uint32_t *d_status, void *stream) {
  // every argument check before any device work
  int rc = check_graph(g, true);
  if (rc || (rc = check_P(P)) || (rc = check_parts(parts)) || (rc = check_local(local)) ||
      (rc = check_contigs(contigs)))
    return rc;
  if (!d_counts || (g->n > 0 && (!flags || !label))) return set_error(CG_EINVAL, "NULL argument");
  if (weight != CG_WEIGHT_READS && weight != CG_WEIGHT_BASES)
    return set_error(CG_EINVAL, "weight=%d is neither CG_WEIGHT_READS nor CG_WEIGHT_BASES", weight);
  const size_t need = layout(g->n, g->m, P).total;
  if (need > (size_t)CG_NOALLOC_SCRATCH_BYTES)
    return set_error(CG_EUNSUPPORTED,
                     "n=%d m=%d P=%d needs %zu bytes of scratch, above the %llu of the "
                     "allocation-free entry point", g->n, g->m, P, need,
                     (unsigned long long)CG_NOALLOC_SCRATCH_BYTES);
  int dev = 0;
  if ((rc = hip_check(hipGetDevice(&dev), "hipGetDevice"))) return rc;
  char *base = nullptr;
  if ((rc = scratch_on(dev, &base))) return rc;
  // a context view of the static array: no events, no allocation
  cg_ctx view{};
  view.device = dev;
  view.fixed = (Fixed *)base;
  view.scratch = base + kFixedBytes;
  view.scratch_bytes = (size_t)CG_NOALLOC_SCRATCH_BYTES;
  view.prof = nullptr;
  Scratch s;
  if (!carve(&view, g->n, g->m, P, &s))
    return set_error(CG_EUNSUPPORTED, "scratch layout does not fit");  // excluded above
  hipStream_t st = (hipStream_t)stream;
  const int n_status = scan_blocks((int64_t)(g->n > 0 ? g->n : 1) + 1) + 1;
  hipLaunchKernelGGL(k_noalloc_reset, dim3(1), dim3(256), 0, st, view.fixed, s.scan_status,
                     n_status);
  if ((rc = hip_check(hipGetLastError(), "k_noalloc_reset"))) return rc;
  rc = launch_mask(&view, *g, flags, d_counts, st);
  if (!rc) rc = launch_components(&view, *g, flags, label, st);
  if (!rc) rc = launch_partition(&view, *g, s, flags, label, P, min_reads, weight, *parts, st);
  if (!rc) rc = launch_induce(&view, *g, s, flags, label, *parts, P, *local, st);
  if (!rc) rc = launch_assemble(&view, *g, s, *parts, *local, P, *contigs, st);
  if (rc) return rc;
  if (d_status) {
    hipLaunchKernelGGL(k_noalloc_status, dim3(1), dim3(1), 0, st, view.fixed, d_status);
    rc = hip_check(hipGetLastError(), "k_noalloc_status");
  }
  return rc;
}
