// Host-only checks of libskm's inputs and the checkpoint file format (see
// host_checks.h).  No HIP here: the library links this file, and a CPU test
// builds it alone under AddressSanitizer and UBSan and feeds it malformed rows
// and truncated or corrupted checkpoints.
#include "host_checks.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

namespace skm {
namespace host {
namespace {

// Checkpoint file: this header, then a int32[n_rows], lo and hi double[n_rows],
// changed uint8[k], and the centroids of the clusters with no members: their
// ids int32[n_empty], row offsets int64[n_empty + 1], terms int32[empty_nnz]
// and values double[empty_nnz].  Every other centroid is the normalised sum of
// its members in ascending row order, a function of the assignment.
struct Header {
  char magic[8];
  uint32_t version;
  int32_t k;
  int64_t n_rows, n_cols, nnz;
  int32_t precision;
  uint32_t flags;
  int32_t iter, last_changed;
  int64_t last_moved;
  int32_t idx_skip, idx_backoff;
  int32_t index_ready, reserved;
  double full_frac;
  int64_t n_empty, empty_nnz;
};
constexpr char kMagic[8] = {'S', 'K', 'M', 'C', 'K', 'P', 'T', '1'};

bool no(std::string *why, const std::string &msg) {
  if (why) *why = msg;
  return false;
}

// Bytes after the header that a header implies, or -1 when its counts are
// out of range (checked without overflow).
int64_t body_bytes(const Header &h) {
  const int64_t N = h.n_rows, k = h.k, ne = h.n_empty, nz = h.empty_nnz;
  if (N < 1 || N > (int64_t(1) << 40) || k < 1 || k > 65535 || ne < 0 || ne > k || nz < 0 ||
      h.n_cols < 1 || h.n_cols > INT32_MAX || nz > ne * h.n_cols)
    return -1;
  return N * (4 + 8 + 8) + k + ne * 4 + (ne + 1) * 8 + nz * (4 + 8);
}

}  // namespace

bool csr_header_ok(const skm_csr *d, int64_t max_cols, bool *unsupported, std::string *why) {
  if (unsupported) *unsupported = false;
  if (!d) return no(why, "docs is NULL");
  if (d->n_rows < 0 || d->n_cols < 1 || d->nnz < 0) return no(why, "bad CSR sizes");
  if (max_cols > 0 && d->n_cols > max_cols) return no(why, "n_cols exceeds the context's vocabulary");
  if (d->n_cols > INT32_MAX || d->n_rows > INT32_MAX) {
    if (unsupported) *unsupported = true;
    return no(why, "n_rows and n_cols must fit int32");
  }
  if (d->n_rows > 0 && (!d->indptr || (d->nnz > 0 && (!d->indices || !d->values))))
    return no(why, "CSR array pointer is NULL");
  return true;
}

bool indptr_ok(const int64_t *ip, int64_t n, int64_t nnz, std::string *why) {
  if (!ip) return no(why, "indptr is NULL");
  if (ip[0] != 0) return no(why, "indptr[0] != 0");
  for (int64_t i = 0; i < n; ++i)
    if (ip[i + 1] < ip[i]) return no(why, "indptr decreases at row " + std::to_string(i));
  if (ip[n] != nnz) return no(why, "indptr[n_rows] != nnz");
  return true;
}

bool rows_ok(const int64_t *ip, const int32_t *ix, const float *v, int64_t n, int64_t nnz,
             int64_t n_cols, std::string *why) {
  if (!indptr_ok(ip, n, nnz, why)) return false;
  if (nnz > 0 && (!ix || !v)) return no(why, "CSR array pointer is NULL");
  for (int64_t i = 0; i < n; ++i) {
    const int64_t b = ip[i], e = ip[i + 1];
    if (e == b) return no(why, "empty row");
    double sq = 0.0;
    for (int64_t q = b; q < e; ++q) {
      const int32_t t = ix[q];
      const float x = v[q];
      if (t < 0 || t >= n_cols) return no(why, "term index out of range");
      if (q > b && t <= ix[q - 1]) return no(why, "indices must be strictly ascending within a row");
      if (!(x > 0.0f) || !std::isfinite(x)) return no(why, "values must be finite and > 0");
      sq += (double)x * (double)x;
    }
    if (std::fabs(std::sqrt(sq) - 1.0) > 1e-5)
      return no(why, "row L2 norm differs from 1 by more than 1e-5");
  }
  return true;
}

bool write_checkpoint(const char *path, const Checkpoint &ck, std::string *why) {
  if (!path) return no(why, "path is NULL");
  Header h{};
  std::memcpy(h.magic, kMagic, 8);
  h.version = 1;
  h.k = ck.k;
  h.n_rows = ck.n_rows;
  h.n_cols = ck.n_cols;
  h.nnz = ck.nnz;
  h.precision = ck.precision;
  h.flags = ck.flags;
  h.iter = ck.iter;
  h.last_changed = ck.last_changed;
  h.last_moved = ck.last_moved;
  h.idx_skip = ck.idx_skip;
  h.idx_backoff = ck.idx_backoff;
  h.index_ready = ck.index_ready;
  h.full_frac = ck.full_frac;
  h.n_empty = (int64_t)ck.e_ids.size();
  h.empty_nnz = (int64_t)ck.e_terms.size();
  if ((int64_t)ck.a.size() != ck.n_rows || (int64_t)ck.lo.size() != ck.n_rows ||
      (int64_t)ck.hi.size() != ck.n_rows || (int64_t)ck.changed.size() != ck.k ||
      ck.e_off.size() != ck.e_ids.size() + 1 || ck.e_vals.size() != ck.e_terms.size())
    return no(why, "inconsistent checkpoint contents");
  // written beside the target and renamed over it, so that a crash while
  // writing leaves the previous checkpoint intact
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "wb");
  if (!f) return no(why, "cannot open " + tmp + " for writing");
  bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1;
  auto put = [&](const void *p, size_t bytes) {
    if (ok && bytes) ok = std::fwrite(p, 1, bytes, f) == bytes;
  };
  put(ck.a.data(), sizeof(int32_t) * ck.a.size());
  put(ck.lo.data(), sizeof(double) * ck.lo.size());
  put(ck.hi.data(), sizeof(double) * ck.hi.size());
  put(ck.changed.data(), ck.changed.size());
  put(ck.e_ids.data(), sizeof(int32_t) * ck.e_ids.size());
  put(ck.e_off.data(), sizeof(int64_t) * ck.e_off.size());
  put(ck.e_terms.data(), sizeof(int32_t) * ck.e_terms.size());
  put(ck.e_vals.data(), sizeof(double) * ck.e_vals.size());
  ok = (std::fflush(f) == 0) && ok;
  ok = (std::fclose(f) == 0) && ok;
  if (ok) ok = std::rename(tmp.c_str(), path) == 0;
  if (!ok) {
    (void)std::remove(tmp.c_str());
    return no(why, std::string("writing ") + path + " failed");
  }
  return true;
}

bool read_checkpoint(const char *path, int64_t n_rows, int64_t n_cols, int64_t nnz,
                     Checkpoint *out, std::string *why) {
  if (!path || !out) return no(why, "path or out is NULL");
  FILE *f = std::fopen(path, "rb");
  if (!f) return no(why, std::string("cannot open ") + path);
  const std::string pre = std::string("checkpoint ") + path + ": ";
  auto bad = [&](const char *msg) {
    std::fclose(f);
    return no(why, pre + msg);
  };
  Header h{};
  if (std::fread(&h, sizeof(h), 1, f) != 1 || std::memcmp(h.magic, kMagic, 8) != 0 ||
      h.version != 1)
    return bad("not a checkpoint of this library");
  if (h.n_rows != n_rows || h.n_cols != n_cols || h.nnz != nnz)
    return bad("taken on rows of another shape");
  const int64_t body = body_bytes(h);
  if (body < 0 || h.k > h.n_rows || h.iter < 1) return bad("inconsistent header");
  // the file must hold exactly what the header announces: nothing is
  // allocated from a count the file cannot back
  if (std::fseek(f, 0, SEEK_END) != 0) return bad("cannot seek");
  const long end = std::ftell(f);
  if (end < 0 || (int64_t)end != (int64_t)sizeof(Header) + body)
    return bad((int64_t)end < (int64_t)sizeof(Header) + body ? "truncated" : "trailing bytes");
  if (std::fseek(f, (long)sizeof(Header), SEEK_SET) != 0) return bad("cannot seek");
  Checkpoint ck;
  ck.k = h.k;
  ck.n_rows = h.n_rows;
  ck.n_cols = h.n_cols;
  ck.nnz = h.nnz;
  ck.precision = h.precision;
  ck.flags = h.flags;
  ck.iter = h.iter;
  ck.last_changed = h.last_changed;
  ck.last_moved = h.last_moved;
  ck.idx_skip = h.idx_skip;
  ck.idx_backoff = h.idx_backoff;
  ck.index_ready = h.index_ready;
  ck.full_frac = h.full_frac;
  const int64_t N = h.n_rows, D = h.n_cols, ne = h.n_empty, nz = h.empty_nnz;
  const int32_t k = h.k;
  try {
    ck.a.resize(N);
    ck.lo.resize(N);
    ck.hi.resize(N);
    ck.changed.resize(k);
    ck.e_ids.resize(ne);
    ck.e_off.resize(ne + 1);
    ck.e_terms.resize(nz);
    ck.e_vals.resize(nz);
  } catch (const std::bad_alloc &) {
    return bad("not enough host memory");
  }
  bool ok = true;
  auto get = [&](void *p, size_t bytes) {
    if (ok && bytes) ok = std::fread(p, 1, bytes, f) == bytes;
  };
  get(ck.a.data(), sizeof(int32_t) * N);
  get(ck.lo.data(), sizeof(double) * N);
  get(ck.hi.data(), sizeof(double) * N);
  get(ck.changed.data(), (size_t)k);
  get(ck.e_ids.data(), sizeof(int32_t) * ne);
  get(ck.e_off.data(), sizeof(int64_t) * (ne + 1));
  get(ck.e_terms.data(), sizeof(int32_t) * nz);
  get(ck.e_vals.data(), sizeof(double) * nz);
  if (!ok) return bad("truncated");
  std::vector<int64_t> count(k, 0);
  for (int32_t j : ck.a) {
    if (j < 0 || j >= k) return bad("assignment out of range");
    count[j] += 1;
  }
  for (int64_t i = 0; i < N; ++i)
    if (!(ck.lo[i] <= ck.hi[i])) return bad("bad certified interval");
  if (ck.e_off[0] != 0 || ck.e_off[ne] != nz) return bad("bad row offsets");
  for (int64_t q = 0; q < ne; ++q) {
    const int32_t j = ck.e_ids[q];
    if (j < 0 || j >= k || count[j] != 0 || (q > 0 && j <= ck.e_ids[q - 1]))
      return bad("bad empty-cluster ids");
    if (ck.e_off[q + 1] < ck.e_off[q] || ck.e_off[q + 1] > nz) return bad("bad row offsets");
    for (int64_t p = ck.e_off[q]; p < ck.e_off[q + 1]; ++p) {
      if (ck.e_terms[p] < 0 || ck.e_terms[p] >= D) return bad("term out of range");
      if (p > ck.e_off[q] && ck.e_terms[p] <= ck.e_terms[p - 1]) return bad("terms not ascending");
      if (!std::isfinite(ck.e_vals[p])) return bad("non-finite centroid value");
    }
  }
  int64_t n_empty_a = 0;
  for (int32_t j = 0; j < k; ++j) n_empty_a += count[j] == 0;
  if (n_empty_a != ne) return bad("empty clusters do not match the assignment");
  std::fclose(f);
  *out = std::move(ck);
  return true;
}

}  // namespace host
}  // namespace skm
