// Driver for the host-side input checks of libskm (host_checks.cpp) under
// AddressSanitizer and UBSan: well-formed rows and checkpoints pass,
// malformed rows, truncated files (every length), corrupted headers and
// corrupted bodies are refused without any out-of-bounds access, overflow or
// oversized allocation.  Prints "host checks ok" when every expectation holds.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../paper_2108_00895_amd/csrc/host_checks.h"

using namespace skm::host;

static int failures = 0;

static void expect(bool cond, const char *what) {
  if (!cond) {
    std::printf("FAILED: %s\n", what);
    ++failures;
  }
}

struct Rows {
  std::vector<int64_t> ip;
  std::vector<int32_t> ix;
  std::vector<float> v;
};

// n rows of 3 terms each, unit length.
static Rows good_rows(int64_t n, int32_t D) {
  Rows r;
  r.ip.push_back(0);
  for (int64_t i = 0; i < n; ++i) {
    for (int32_t q = 0; q < 3; ++q) {
      r.ix.push_back((int32_t)((i + 5 * q) % D));
      r.v.push_back((float)(1.0 / std::sqrt(3.0)));
    }
    // keep the row's terms ascending
    int32_t *t = r.ix.data() + r.ix.size() - 3;
    for (int a = 0; a < 3; ++a)
      for (int b = a + 1; b < 3; ++b)
        if (t[b] < t[a]) std::swap(t[a], t[b]);
    r.ip.push_back((int64_t)r.ix.size());
  }
  return r;
}

static bool rows_ok_(const Rows &r, int32_t D) {
  std::string why;
  return rows_ok(r.ip.data(), r.ix.data(), r.v.data(), (int64_t)r.ip.size() - 1,
                 (int64_t)r.ix.size(), D, &why);
}

static void check_rows() {
  const int32_t D = 40;
  Rows g = good_rows(20, D);
  expect(rows_ok_(g, D), "good rows pass");
  {
    Rows r = g;
    r.ip[0] = 1;
    expect(!rows_ok_(r, D), "indptr[0] != 0");
  }
  {
    Rows r = g;
    r.ip[5] = r.ip[6] + 1;
    expect(!rows_ok_(r, D), "decreasing indptr");
  }
  {
    Rows r = g;
    r.ip.back() += 1;
    expect(!rows_ok_(r, D), "indptr[n] != nnz");
  }
  {
    Rows r = g;
    r.ix[4] = D;
    expect(!rows_ok_(r, D), "term out of range");
  }
  {
    Rows r = g;
    r.ix[4] = -1;
    expect(!rows_ok_(r, D), "negative term");
  }
  {
    Rows r = g;
    std::swap(r.ix[3], r.ix[4]);
    expect(!rows_ok_(r, D), "terms not ascending");
  }
  {
    Rows r = g;
    r.v[7] = 0.0f;
    expect(!rows_ok_(r, D), "zero value");
  }
  {
    Rows r = g;
    r.v[7] = std::nanf("");
    expect(!rows_ok_(r, D), "NaN value");
  }
  {
    Rows r = g;
    r.v[7] = INFINITY;
    expect(!rows_ok_(r, D), "infinite value");
  }
  {
    Rows r = g;
    r.v[7] *= 1.01f;
    expect(!rows_ok_(r, D), "row not unit length");
  }
  {
    Rows r = g;
    r.ip.insert(r.ip.begin() + 3, r.ip[3]);   // an empty row
    expect(!rows_ok_(r, D), "empty row");
  }
  std::string why;
  bool uns = false;
  expect(!csr_header_ok(nullptr, 0, &uns, &why), "NULL docs");
  skm_csr d{10, D, 30, g.ip.data(), g.ix.data(), g.v.data(), 0};
  expect(csr_header_ok(&d, 0, &uns, &why), "good header");
  d.n_rows = -1;
  expect(!csr_header_ok(&d, 0, &uns, &why), "negative rows");
  d.n_rows = 10;
  expect(!csr_header_ok(&d, D - 1, &uns, &why), "too many columns");
  d.n_cols = (int64_t)1 << 33;
  expect(!csr_header_ok(&d, 0, &uns, &why) && uns, "columns beyond int32: unsupported");
  d.n_cols = D;
  d.indices = nullptr;
  expect(!csr_header_ok(&d, 0, &uns, &why), "NULL indices");
}

static Checkpoint good_ckpt() {
  Checkpoint ck;
  ck.k = 5;
  ck.n_rows = 50;
  ck.n_cols = 40;
  ck.nnz = 150;
  ck.precision = 1;
  ck.flags = 3;
  ck.iter = 7;
  ck.last_changed = 2;
  ck.last_moved = 4;
  ck.idx_backoff = 8;
  ck.full_frac = 0.25;
  for (int64_t i = 0; i < ck.n_rows; ++i) {
    ck.a.push_back((int32_t)(i % 4));   // cluster 4 has no members
    ck.lo.push_back(0.5);
    ck.hi.push_back(0.6);
  }
  ck.changed = {1, 0, 0, 1, 0};
  ck.e_ids = {4};
  ck.e_off = {0, 3};
  ck.e_terms = {2, 9, 30};
  ck.e_vals = {0.5, 0.5, std::sqrt(0.5)};
  return ck;
}

static std::vector<unsigned char> slurp(const std::string &p) {
  std::vector<unsigned char> b;
  FILE *f = std::fopen(p.c_str(), "rb");
  if (!f) return b;
  int c;
  while ((c = std::fgetc(f)) != EOF) b.push_back((unsigned char)c);
  std::fclose(f);
  return b;
}

static void spit(const std::string &p, const std::vector<unsigned char> &b) {
  FILE *f = std::fopen(p.c_str(), "wb");
  if (!f) return;
  if (!b.empty()) std::fwrite(b.data(), 1, b.size(), f);
  std::fclose(f);
}

static bool read_(const std::string &p, Checkpoint *out) {
  std::string why;
  return read_checkpoint(p.c_str(), 50, 40, 150, out, &why);
}

template <typename T>
static void poke(std::vector<unsigned char> &b, size_t off, T val) {
  std::memcpy(b.data() + off, &val, sizeof(T));
}

static void check_checkpoints(const std::string &dir) {
  const std::string p = dir + "/ck.bin", q = dir + "/bad.bin";
  std::string why;
  Checkpoint ck = good_ckpt();
  expect(write_checkpoint(p.c_str(), ck, &why), "write");
  Checkpoint back;
  expect(read_(p, &back), "read back");
  expect(back.a == ck.a && back.lo == ck.lo && back.hi == ck.hi && back.changed == ck.changed &&
             back.e_ids == ck.e_ids && back.e_off == ck.e_off && back.e_terms == ck.e_terms &&
             back.e_vals == ck.e_vals && back.iter == ck.iter && back.full_frac == ck.full_frac,
         "round trip");
  std::string w2;
  expect(!read_checkpoint(p.c_str(), 51, 40, 150, &back, &w2), "other shape refused");
  const std::vector<unsigned char> good = slurp(p);
  // every truncation, and a trailing byte
  for (size_t len = 0; len < good.size(); ++len) {
    spit(q, std::vector<unsigned char>(good.begin(), good.begin() + len));
    if (read_(q, &back)) {
      std::printf("FAILED: truncated to %zu bytes accepted\n", len);
      ++failures;
    }
  }
  {
    std::vector<unsigned char> b = good;
    b.push_back(0);
    spit(q, b);
    expect(!read_(q, &back), "trailing byte refused");
  }
  // header fields (offsets follow the header's layout): k, n_empty and
  // empty_nnz huge or negative, iter 0, bad magic and version
  const size_t off_k = 12, off_iter = 48, off_ne = 88, off_nz = 96;
  struct H {
    size_t off;
    int64_t val;
    int width;
    const char *what;
  } hs[] = {{off_k, 70000, 4, "k beyond 65535"},      {off_k, -3, 4, "negative k"},
            {off_k, 60, 4, "k above n_rows"},          {off_iter, 0, 4, "iteration 0"},
            {off_ne, 1ll << 40, 8, "huge n_empty"},    {off_ne, -1, 8, "negative n_empty"},
            {off_nz, 1ll << 45, 8, "huge empty_nnz"},  {off_nz, -5, 8, "negative empty_nnz"},
            {off_nz, 4, 8, "empty_nnz off by one"},    {0, 0, 8, "bad magic"},
            {8, 2, 4, "bad version"}};
  for (const H &h : hs) {
    std::vector<unsigned char> b = good;
    if (h.width == 4)
      poke<int32_t>(b, h.off, (int32_t)h.val);
    else
      poke<int64_t>(b, h.off, h.val);
    spit(q, b);
    expect(!read_(q, &back), h.what);
  }
  // body: an assignment out of range, a member in the listed empty cluster,
  // offsets and terms out of range, an inverted interval
  const size_t hdr = 104, N = 50, k = 5;
  const size_t off_a = hdr, off_lo = off_a + 4 * N, off_ch = off_lo + 16 * N;
  const size_t off_eid = off_ch + k, off_eoff = off_eid + 4, off_term = off_eoff + 16;
  {
    std::vector<unsigned char> b = good;
    poke<int32_t>(b, off_a + 4 * 7, 9);
    spit(q, b);
    expect(!read_(q, &back), "assignment out of range");
  }
  {
    std::vector<unsigned char> b = good;
    poke<int32_t>(b, off_a + 4 * 7, 4);
    spit(q, b);
    expect(!read_(q, &back), "listed empty cluster has a member");
  }
  {
    std::vector<unsigned char> b = good;
    poke<int32_t>(b, off_eid, 7);
    spit(q, b);
    expect(!read_(q, &back), "empty-cluster id out of range");
  }
  {
    std::vector<unsigned char> b = good;
    poke<int64_t>(b, off_eoff + 8, 2);
    spit(q, b);
    expect(!read_(q, &back), "last offset short of empty_nnz");
  }
  {
    std::vector<unsigned char> b = good;
    poke<int64_t>(b, off_eoff, -1);
    spit(q, b);
    expect(!read_(q, &back), "first offset negative");
  }
  {
    std::vector<unsigned char> b = good;
    poke<int32_t>(b, off_term + 4, 99);
    spit(q, b);
    expect(!read_(q, &back), "term out of range");
  }
  {
    std::vector<unsigned char> b = good;
    poke<double>(b, off_lo + 8 * 3, 0.9);
    spit(q, b);
    expect(!read_(q, &back), "lower bound above upper bound");
  }
  expect(!read_(dir + "/missing.bin", &back), "missing file");
  std::remove(p.c_str());
  std::remove(q.c_str());
}

int main(int argc, char **argv) {
  const std::string dir = argc > 1 ? argv[1] : ".";
  check_rows();
  check_checkpoints(dir);
  if (failures) {
    std::printf("%d expectation(s) failed\n", failures);
    return 1;
  }
  std::printf("host checks ok\n");
  return 0;
}
