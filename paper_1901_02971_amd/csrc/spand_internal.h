// Internal structures of libspand: the symbolic analysis (host) shared by the
// factorization and solve drivers.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "spand.h"

namespace spand {

// Separator id (level l, index k), packed as l * 2^32 + k; 0 = none.
inline int64_t sep_pack(int64_t l, int64_t k) { return (l << 32) | k; }
inline int64_t sep_level(int64_t c) { return c >> 32; }
inline int64_t sep_index(int64_t c) { return c & 0xffffffffLL; }
// Ancestor at level l of an id deeper than l; other ids unchanged.
inline int64_t sep_truncate(int64_t c, int64_t l) {
  if (c == 0) return 0;
  int64_t a = sep_level(c);
  if (a <= l) return c;
  return sep_pack(l, ((sep_index(c) - 1) >> (a - l)) + 1);
}

inline uint64_t pair_pack(int32_t i, int32_t j) { return (uint64_t(uint32_t(i)) << 32) | uint32_t(j); }
inline int32_t pair_i(uint64_t p) { return int32_t(p >> 32); }
inline int32_t pair_j(uint64_t p) { return int32_t(p & 0xffffffffu); }

// One elimination step of the symbolic factorization.  Clusters are numbered in
// the canonical order (separator level descending, separator index, left pointer,
// right pointer); those of the eliminated level come first (ids 0..ne-1).
struct SymStep {
  int32_t level = 0;
  int32_t nc = 0;
  int32_t ne = 0;
  std::vector<int64_t> key;        // 3*nc: S, L, R (truncated to `level`)
  std::vector<int64_t> child_ptr;  // nc+1
  std::vector<int32_t> child;      // step 1: vertex ids; later: previous-step cluster ids
  std::vector<uint64_t> before;    // blocks (i >= j) before elimination, sorted
  std::vector<uint64_t> after;     // blocks among remaining clusters after fill, sorted
  std::vector<int64_t> enb_ptr;    // ne+1: neighbours of eliminated clusters
  std::vector<int32_t> enb;
  std::vector<int64_t> nb_ptr;     // nc+1: neighbours (after fill) of remaining clusters
  std::vector<int32_t> nb;
  std::vector<int32_t> colour;     // nc (-1 for eliminated)
  std::vector<int32_t> parent;     // nc (-1 if eliminated or no next step)
};

struct Analysis {
  int64_t n = 0;
  int32_t levels = 0;
  int32_t dim = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> colind;
  std::vector<double> coords;
  std::vector<int64_t> S, L, R;
  std::vector<SymStep> steps;
};

// Kernel-shape and path parameters of a handle before any tuning.
inline spand_tuning default_tuning() {
  spand_tuning t{};
  t.chol_group = 3;
  t.fuse128_min = 256;
  t.gemm_syrk = 0;
  t.gemm_chol = 0;
  t.gemm_scale = 0;
  return t;
}

// Runs Algorithm 2 and the symbolic factorization; returns an error text or "".
std::string analyze_pattern(Analysis& an);

}  // namespace spand
