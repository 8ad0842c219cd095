// skm_assign_new_static: the new-row assignment of skm_assign_new for callers
// that cannot allocate device memory.  Its temporaries (per-row norms, chunk
// partials, certified intervals, the exact tier's row lists and counters) live
// in one fixed device array of this library, `scratch`; the rows are read in
// place from the caller's device CSR and the answers written straight into the
// caller's device outputs.  Nothing here calls hipMalloc or hipFree.
//
// Each GPU holds its own copy of `scratch`.  Its device address is looked up
// once per device with hipGetSymbolAddress (at skm_init, with the context's
// device current) and kept; host code never passes the array's own name to a
// kernel.  Calls on one GPU share that GPU's copy, so calls that overlap on the
// same GPU race: callers serialise them (one stream, or their own lock).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per GPU

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::vector<unsigned char *> g_addr;   // per device id, nullptr until looked up

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of one call's temporaries for n rows and nch chunks.
struct Layout {
  size_t xl1, xl2, part, lo, hi, flag_L, flag_rows, flag_mode, counters, stat, bad, total;
};

Layout layout(int64_t n, int64_t nch) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.xl1 = take(8 * (size_t)n);
  L.xl2 = take(8 * (size_t)n);
  L.part = take(sizeof(skm::Partial) * (size_t)nch * (size_t)n);
  L.lo = take(8 * (size_t)n);
  L.hi = take(8 * (size_t)n);
  L.flag_L = take(8 * (size_t)n);
  L.flag_rows = take(4 * (size_t)n);
  L.flag_mode = take((size_t)n);
  L.counters = take(8 * sizeof(int32_t));
  L.stat = take(16 * sizeof(unsigned long long));
  L.bad = take(sizeof(int32_t));
  L.total = o;
  return L;
}

}  // namespace

namespace skm {

// Looks up (once per device) the device address of `scratch` on the current
// device, which must be `device`.
skm_status noalloc_setup(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device < 0) return set_error(SKM_E_INVALID, "bad device id");
  if ((size_t)device < g_addr.size() && g_addr[device]) return SKM_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return set_error(SKM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                       hipGetErrorString(e));
  }
  if (g_addr.size() <= (size_t)device) g_addr.resize(device + 1, nullptr);
  g_addr[device] = static_cast<unsigned char *>(p);
  return SKM_OK;
}

}  // namespace skm

extern "C" {

size_t skm_static_scratch_bytes(void) { return kScratchBytes; }

int64_t skm_static_max_rows(const skm_ctx *c) {
  if (!c) return 0;
  const int64_t nch = ((int64_t)c->k + skm::kChunk - 1) / skm::kChunk;
  // layout() takes 45 + 32 nch bytes per row plus at most 255 bytes of
  // padding for each of its 11 pieces
  const int64_t per_row = 8 * 5 + 4 + 1 + (int64_t)sizeof(skm::Partial) * nch;
  int64_t n = (int64_t)(kScratchBytes - 12 * 256) / per_row;
  while (n > 0 && layout(n, nch).total > kScratchBytes) --n;
  return n;
}

skm_status skm_assign_new_static(skm_ctx *c, const skm_csr *docs, int32_t *out_assign,
                                 double *out_score, void *stream) {
  using namespace skm;
  if (!c) return set_error(SKM_E_INVALID, "context is NULL");
  if (c->poisoned) return set_error(SKM_E_DEVICE, "context is poisoned by an earlier device error");
  if (!docs) return set_error(SKM_E_INVALID, "docs is NULL");
  if (!docs->on_device)
    return set_error(SKM_E_INVALID, "skm_assign_new_static takes device rows (on_device = 1)");
  const int64_t n = docs->n_rows, z = docs->nnz;
  if (n < 0 || z < 0 || docs->n_cols < 1 || docs->n_cols > c->D)
    return set_error(SKM_E_INVALID, "bad CSR sizes");
  if (n == 0) return SKM_OK;
  if (!docs->indptr || (z > 0 && (!docs->indices || !docs->values)))
    return set_error(SKM_E_INVALID, "CSR array pointer is NULL");
  if (!out_assign || !out_score) return set_error(SKM_E_INVALID, "output pointer is NULL");
  const int64_t max_rows = skm_static_max_rows(c);
  if (n > max_rows)
    return set_error(SKM_E_INVALID, "n_rows " + std::to_string(n) + " exceeds the " +
                                        std::to_string(max_rows) + " rows that the " +
                                        std::to_string(kScratchBytes >> 20) +
                                        " MiB static workspace holds at k = " +
                                        std::to_string(c->k));
  unsigned char *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if ((size_t)c->device < g_addr.size()) base = g_addr[c->device];
  }
  if (!base) return set_error(SKM_E_STATE, "static workspace not set up on this device");
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;

  // indptr is checked on the host before any kernel walks the rows
  std::vector<int64_t> ip(n + 1);
  hipError_t e = hipMemcpyAsync(ip.data(), docs->indptr, sizeof(int64_t) * (n + 1),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    c->poisoned = true;
    return set_error(SKM_E_DEVICE, std::string("reading indptr: ") + hipGetErrorString(e));
  }
  if (ip[0] != 0 || ip[n] != z) return set_error(SKM_E_INVALID, "indptr[0] != 0 or indptr[n] != nnz");
  for (int64_t i = 0; i < n; ++i)
    if (ip[i + 1] < ip[i]) return set_error(SKM_E_INVALID, "indptr decreases");

  const int64_t nch = ((int64_t)c->k + kChunk - 1) / kChunk;
  const Layout L = layout(n, nch);
  double *xl1 = reinterpret_cast<double *>(base + L.xl1);
  double *xl2 = reinterpret_cast<double *>(base + L.xl2);
  int32_t *bad = reinterpret_cast<int32_t *>(base + L.bad);
  int32_t hbad = 0;
  e = launch_fill_i32(bad, 0, 1, s);
  if (e == hipSuccess)
    e = launch_row_stats(docs->indptr, docs->indices, docs->values, n, c->D, xl1, xl2, bad, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    c->poisoned = true;
    return set_error(SKM_E_DEVICE, std::string("row checks: ") + hipGetErrorString(e));
  }
  if (hbad & 4) return set_error(SKM_E_INVALID, "term index out of range [0, n_cols)");
  if (hbad & 2) return set_error(SKM_E_INVALID, "values must be finite and > 0");
  if (hbad & 8) return set_error(SKM_E_INVALID, "indices must be strictly ascending within a row");
  if (hbad & 32) return set_error(SKM_E_INVALID, "empty row");
  if (hbad & 16) return set_error(SKM_E_INVALID, "row L2 norm differs from 1 by more than 1e-5");

  NewRows nr{docs->indptr,
             docs->indices,
             docs->values,
             xl1,
             reinterpret_cast<Partial *>(base + L.part),
             out_assign,
             reinterpret_cast<double *>(base + L.lo),
             reinterpret_cast<double *>(base + L.hi),
             reinterpret_cast<int32_t *>(base + L.flag_rows),
             reinterpret_cast<double *>(base + L.flag_L),
             base + L.flag_mode,
             reinterpret_cast<int32_t *>(base + L.counters),
             reinterpret_cast<unsigned long long *>(base + L.stat),
             out_score};
  e = launch_new_rows(c, nr, n, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    c->poisoned = true;
    return set_error(SKM_E_DEVICE, std::string("skm_assign_new_static: ") + hipGetErrorString(e));
  }
  return SKM_OK;
}

}  // extern "C"
