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
__global__ void __launch_bounds__(WG) k_reduce(const ReduceDesc* __restrict__ descs,
                                               const ContribDesc* __restrict__ cs) {
  const ReduceDesc d = descs[blockIdx.x];
  const uint32_t rows = (uint32_t)d.rows;
  for (uint32_t e = (uint32_t)d.e0 + threadIdx.x; e < (uint32_t)d.e1; e += WG) {
    const uint32_t c = e / rows, r = e - c * rows;
    if (d.diag && r < c) continue;
    double sum = 0.0;
    for (int q = d.c_begin; q < d.c_end; ++q) {
      const ContribDesc cd = cs[q];
      sum += cd.C[r + (int64_t)c * cd.ldC];
    }
    d.T[r + (int64_t)c * d.ldT] -= sum;
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
__global__ void __launch_bounds__(WG) k_copy(const CopyDesc* __restrict__ descs) {
  const CopyDesc d = descs[blockIdx.x];
  const int h = min(d.rows, WG), cs = WG / h;
  const int r0 = threadIdx.x % h, dc = threadIdx.x / h;
  if (dc >= cs) return;
  for (int c = d.c0 + dc; c < d.c1; c += cs)
    for (int r = r0; r < d.rows; r += h)
      d.dst[r + (int64_t)c * d.ldd] = d.trans ? d.src[c + (int64_t)r * d.lds] : d.src[r + (int64_t)c * d.lds];
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

}  // namespace spand
