// Host-only checks of libskm's inputs: the CSR conventions of skm.h and the
// checkpoint file (read and written here).  Plain C++ (no HIP), so that these
// parsers of caller-supplied data can be built and exercised under
// AddressSanitizer and UBSan on the host alone.  Each function returns true on
// success and otherwise stores the reason in *why.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "skm.h"

namespace skm {
namespace host {

// Shape and pointers of a CSR description (not its contents).  max_cols > 0:
// n_cols must not exceed it.  *unsupported is set when the sizes are valid but
// outside what the library takes (n_rows or n_cols beyond int32).
bool csr_header_ok(const skm_csr *d, int64_t max_cols, bool *unsupported, std::string *why);

// indptr[0] = 0, non-decreasing, indptr[n] = nnz.
bool indptr_ok(const int64_t *ip, int64_t n, int64_t nnz, std::string *why);

// Every convention of skm.h on host arrays: indptr as above, terms strictly
// ascending within a row and in [0, n_cols), values finite and > 0, no empty
// row, each row's L2 norm within 1e-5 of 1.
bool rows_ok(const int64_t *ip, const int32_t *ix, const float *v, int64_t n, int64_t nnz,
             int64_t n_cols, std::string *why);

// Checkpoint file contents (skm_save / skm_load).
struct Checkpoint {
  int32_t k = 0;
  int64_t n_rows = 0, n_cols = 0, nnz = 0;
  int32_t precision = 0;
  uint32_t flags = 0;
  int32_t iter = 0, last_changed = 0;
  int64_t last_moved = 0;
  int32_t idx_skip = 0, idx_backoff = 0;
  int32_t index_ready = 0;
  double full_frac = 0.0;
  std::vector<int32_t> a;          // [n_rows] assignment that made the centroids
  std::vector<double> lo, hi;      // [n_rows] certified intervals
  std::vector<uint8_t> changed;    // [k]
  std::vector<int32_t> e_ids;      // clusters without members, ascending
  std::vector<int64_t> e_off;      // [n_empty + 1] offsets into e_terms / e_vals
  std::vector<int32_t> e_terms;    // their non-zero terms
  std::vector<double> e_vals;      // and values
};

// Writes the file as path + ".tmp" and renames it to path.
bool write_checkpoint(const char *path, const Checkpoint &ck, std::string *why);

// Reads and checks a whole file before anything is allocated from its
// contents: magic and version, the shape against (n_rows, n_cols, nnz), the
// exact file length the header implies, every id and offset in range, and the
// clusters without members equal to those of the saved assignment.
bool read_checkpoint(const char *path, int64_t n_rows, int64_t n_cols, int64_t nnz,
                     Checkpoint *out, std::string *why);

}  // namespace host
}  // namespace skm
