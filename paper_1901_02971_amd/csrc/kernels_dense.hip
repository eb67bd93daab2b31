// Dense batched kernels of the factorization (gfx950, wave64).
//
//  * k_reduce     deterministic Schur-complement accumulation: every target block
//                 subtracts its contributions in ascending eliminated-cluster order
//                 (one workgroup per range of at most REDUCE_CHUNK entries).
//  * k_copy       strided (optionally transposed) block copies for the merge (Sec. 2.7).
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace spand {

#define WG 256

// Accesses through the global address space: flat accesses also count against the
// LDS counter, and the compiler then waits for every store before the next one.
typedef __attribute__((address_space(1))) const double gdouble_r;
typedef __attribute__((address_space(1))) double gdouble_d;
__device__ inline double gldd(const double* p) { return *(gdouble_r*)p; }
__device__ inline void gstd(double* p, double v) { *(gdouble_d*)p = v; }

// ---------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline int wave_min_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
// Block-wide reductions (blockDim.x == WG); `red` is WG/64 doubles of LDS.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < WG / 64; ++q) s += red[q];
  return s;
}
__device__ inline double block_max(double v, double* red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
  for (int q = 1; q < WG / 64; ++q) s = fmax(s, red[q]);
  return s;
}
__device__ inline int block_min_i(int v, int* red) {
  v = wave_min_i(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  int s = red[0];
  for (int q = 1; q < WG / 64; ++q) s = min(s, red[q]);
  return s;
}

// ---------------------------------------------------------------- CSR scatter
__global__ void k_scatter_values(const double* __restrict__ vals, const int64_t* __restrict__ dst, int64_t nnz,
                                 double* __restrict__ arena, double* __restrict__ elim, int32_t* flag) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  double v = vals[e];
  if (!isfinite(v)) atomicOr(flag, 1);
  int64_t d = dst[e];
  if (d >= 0) arena[d] = v;
  else if (d <= -2) elim[-d - 2] = v;
}

void launch_scatter_values(const double* vals, const int64_t* dst, int64_t nnz, double* arena, double* elim,
                           int32_t* flag, hipStream_t s) {
  if (nnz == 0) return;
  hipLaunchKernelGGL(k_scatter_values, dim3((nnz + 255) / 256), dim3(256), 0, s, vals, dst, nnz, arena, elim, flag);
}

// ---------------------------------------------------------------- Schur reduce
// Only the lower triangle of a diagonal target block is accumulated: its upper
// triangle is never read again (Cholesky, the left solves, the merge and the CPQR
// read lower triangles and off-diagonal blocks only).
// A thread takes RU entries at a time and reads all their contributions and target
// values before it stores any: the target and the contributions may alias as far as
// the compiler knows, so an interleaved loop would wait for every store.  Entries
// outside the range read the first entry of the block and are not stored.
#define RU 8
__global__ void __launch_bounds__(WG) k_reduce(const ReduceDesc* __restrict__ descs,
                                               const ContribDesc* __restrict__ cs) {
  const ReduceDesc d = descs[blockIdx.x];
  const uint32_t rows = (uint32_t)d.rows;
  for (uint32_t eb = (uint32_t)d.e0 + threadIdx.x; eb < (uint32_t)d.e1; eb += WG * RU) {
    bool ok[RU];
    uint32_t rr[RU], cc[RU];
    double sum[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const uint32_t e = eb + u * WG;
      const uint32_t c = e / rows, r = e - c * rows;
      ok[u] = e < (uint32_t)d.e1 && !(d.diag && r < c);
      rr[u] = ok[u] ? r : 0;
      cc[u] = ok[u] ? c : 0;
      sum[u] = 0.0;
    }
    for (int q = d.c_begin; q < d.c_end; ++q) {
      const ContribDesc cd = cs[q];
#pragma unroll
      for (int u = 0; u < RU; ++u) sum[u] += gldd(cd.C + rr[u] + (int64_t)cc[u] * cd.ldC);
    }
    double tv[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) tv[u] = gldd(d.T + rr[u] + (int64_t)cc[u] * d.ldT);
#pragma unroll
    for (int u = 0; u < RU; ++u)
      if (ok[u]) gstd(d.T + rr[u] + (int64_t)cc[u] * d.ldT, tv[u] - sum[u]);
  }
}

void launch_reduce(const ReduceDesc* d, int32_t count, const ContribDesc* c, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_reduce, dim3(count), dim3(WG), 0, s, d, c);
}

// ---------------------------------------------------------------- copies
// One workgroup per column range of a block.  Thread t takes row t % h of column
// c0 + t / h, h = min(rows, WG), and steps by WG / h columns (one division per
// thread, none per entry).
// Entries are moved RU at a time, all loads before the stores (source and
// destination may alias as far as the compiler knows); a slot past the range reads
// the first entry of the source and is not stored.
__global__ void __launch_bounds__(WG) k_copy(const CopyDesc* __restrict__ descs) {
  const CopyDesc d = descs[blockIdx.x];
  const int h = min(d.rows, WG), cs = WG / h;
  const int r0 = threadIdx.x % h, dc = threadIdx.x / h;
  if (dc >= cs) return;
  int c = d.c0 + dc, r = r0;
  while (c < d.c1) {
    bool ok[RU];
    int64_t to[RU];
    double v[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      ok[u] = c < d.c1;
      const int64_t so = ok[u] ? (d.trans ? c + (int64_t)r * d.lds : r + (int64_t)c * d.lds) : 0;
      to[u] = r + (int64_t)c * d.ldd;
      v[u] = gldd(d.src + so);
      r += h;
      if (r >= d.rows) {
        r = r0;
        c += cs;
      }
    }
#pragma unroll
    for (int u = 0; u < RU; ++u)
      if (ok[u]) gstd(d.dst + to[u], v[u]);
  }
}

void launch_copy(const CopyDesc* d, int64_t count, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_copy, dim3(count), dim3(WG), 0, s, d);
}

__global__ void __launch_bounds__(WG) k_set_identity(const IdentDesc* __restrict__ descs) {
  const IdentDesc d = descs[blockIdx.x];
  const int h = min(d.n, WG), cs = WG / h;
  const int r0 = threadIdx.x % h, dc = threadIdx.x / h;
  if (dc >= cs) return;
  for (int c = d.c0 + dc; c < d.c1; c += cs)
    for (int r = r0; r < d.n; r += h) d.D[r + (int64_t)c * d.ld] = (r == c) ? 1.0 : 0.0;
}

void launch_set_identity(const IdentDesc* d, int32_t count, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_set_identity, dim3(count), dim3(WG), 0, s, d);
}

// Zero fill of ranges of at most ZERO_CHUNK doubles, one workgroup each (the step
// buffers of every problem of a factorization run in one launch).
__global__ void __launch_bounds__(WG) k_zero(const ZeroDesc* __restrict__ descs) {
  const ZeroDesc d = descs[blockIdx.x];
  for (int64_t i = threadIdx.x; i < d.len; i += WG) d.p[i] = 0.0;
}

void launch_zero(const ZeroDesc* d, int64_t count, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_zero, dim3(count), dim3(WG), 0, s, d);
}

__global__ void __launch_bounds__(WG) k_remap(const RemapSeg* __restrict__ d, const int32_t* __restrict__ pos) {
  const RemapSeg g = d[blockIdx.x];
  for (int64_t k = threadIdx.x; k < g.len; k += WG) g.p[k] = pos[g.p[k]];
}

void launch_remap(const RemapSeg* d, int64_t count, const int32_t* pos, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_remap, dim3(unsigned(count)), dim3(WG), 0, s, d, pos);
}

// pos[inv[k]] = k on pos filled with -1 beforehand; an entry of inv outside [0, n)
// or met twice sets bit 0 of *bad (inv is then no permutation).
__global__ void __launch_bounds__(WG) k_invert_perm(const int32_t* __restrict__ inv, int64_t n, int32_t* pos,
                                                    int32_t* bad) {
  const int64_t k = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (k >= n) return;
  const int32_t v = inv[k];
  if (v < 0 || v >= n) {
    atomicOr(bad, 1);
    return;
  }
  if (atomicExch(pos + v, (int32_t)k) != -1) atomicOr(bad, 1);
}

void launch_invert_perm(const int32_t* inv, int64_t n, int32_t* pos, int32_t* bad, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_invert_perm, dim3(unsigned((n + WG - 1) / WG)), dim3(WG), 0, s, inv, n, pos, bad);
}

}  // namespace spand
