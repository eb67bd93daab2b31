// Host driver of the analysis (Algorithm 2 + symbolic factorization) for a build of
// csrc/analyze.cpp under AddressSanitizer and UndefinedBehaviorSanitizer: 5/7-point
// grid patterns, with and without coordinates, at several depths; prints one line
// per case with the cluster count of every step.
#include <cstdio>
#include <string>
#include <vector>

#include "spand_internal.h"

static void grid(int nx, int ny, int nz, bool coords, int levels) {
  spand::Analysis an;
  const int64_t n = int64_t(nx) * ny * nz;
  an.n = n;
  an.levels = levels;
  an.dim = coords ? (nz > 1 ? 3 : 2) : 0;
  an.rowptr.assign(n + 1, 0);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int64_t v = i + int64_t(nx) * (j + int64_t(ny) * k);
        std::vector<int32_t> nb;
        if (k > 0) nb.push_back(int32_t(v - int64_t(nx) * ny));
        if (j > 0) nb.push_back(int32_t(v - nx));
        if (i > 0) nb.push_back(int32_t(v - 1));
        nb.push_back(int32_t(v));
        if (i + 1 < nx) nb.push_back(int32_t(v + 1));
        if (j + 1 < ny) nb.push_back(int32_t(v + nx));
        if (k + 1 < nz) nb.push_back(int32_t(v + int64_t(nx) * ny));
        an.colind.insert(an.colind.end(), nb.begin(), nb.end());
        an.rowptr[v + 1] = int64_t(an.colind.size());
        if (coords) {
          an.coords.push_back(i);
          an.coords.push_back(j);
          if (nz > 1) an.coords.push_back(k);
        }
      }
  const std::string err = spand::analyze_pattern(an);
  std::printf("%dx%dx%d L=%d %s: %s", nx, ny, nz, levels, coords ? "rcb" : "graph", err.empty() ? "ok" : err.c_str());
  for (const spand::SymStep& st : an.steps) std::printf(" %d/%d", st.ne, st.nc);
  std::printf("\n");
}

int main() {
  for (bool c : {true, false}) {
    grid(7, 7, 1, c, 3);
    grid(1, 1, 1, c, 1);
    grid(3, 2, 1, c, 4);
    grid(16, 9, 1, c, 5);
    grid(9, 7, 6, c, 4);
    grid(12, 12, 12, c, 6);
    grid(20, 3, 17, c, 7);
  }
  return 0;
}
