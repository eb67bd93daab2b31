// Dense batched kernels of the factorization (gfx950, wave64).
//
//  * k_gemm       batched variable-size GEMM over a flat list of 64x64 output tiles;
//                 carries the trailing updates of the blocked Cholesky, the SYRK of
//                 the Schur update (Sec. 2.4) and the left scaling of Sec. 2.5.
//  * k_reduce     deterministic Schur-complement accumulation: every target block
//                 subtracts its contributions in ascending eliminated-cluster order.
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

// ---------------------------------------------------------------- batched GEMM
// 64x64 output tile per workgroup, 256 threads as 16x16, 4x4 outputs each
// (rows ty + 16*a, columns tx + 16*b), K staged through LDS 16 at a time.
// prec 0: FP64 multiply-add; prec 1: operands rounded to FP32, FP32 products and
// FP32 accumulation (the result is stored to the FP64 target).
template <typename T>
__global__ void __launch_bounds__(WG) k_gemm(const GemmDesc* __restrict__ descs, const TileRef* __restrict__ tiles) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN + 1];
  const TileRef tr = tiles[blockIdx.x];
  const GemmDesc d = descs[tr.desc];
  const int m0 = tr.tm * BM, n0 = tr.tn * BN;
  const bool ta = d.flags & G_TA, tb = d.flags & G_TB;
  int kmax = d.K;
  if (d.flags & G_TRIA) kmax = min(kmax, m0 + BM);
  if (d.flags & G_TRIB) kmax = min(kmax, n0 + BN);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = T(0);
  for (int k0 = 0; k0 < kmax; k0 += BK) {
    // load op(A)[m0:m0+64, k0:k0+16] and op(B)[k0:k0+16, n0:n0+64]
#pragma unroll
    for (int q = 0; q < (BM * BK) / WG; ++q) {
      const int e = threadIdx.x + q * WG;
      int mm, kk;
      if (!ta) { mm = e & 63; kk = e >> 6; } else { kk = e & 15; mm = e >> 4; }
      const int gm = m0 + mm, gk = k0 + kk;
      double v = 0.0;
      if (gm < d.M && gk < kmax && !((d.flags & G_TRIA) && gk > gm))
        v = ta ? d.A[gk + (int64_t)gm * d.lda] : d.A[gm + (int64_t)gk * d.lda];
      As[kk][mm] = T(v);
    }
#pragma unroll
    for (int q = 0; q < (BN * BK) / WG; ++q) {
      const int e = threadIdx.x + q * WG;
      int nn, kk;
      if (!tb) { kk = e & 15; nn = e >> 4; } else { nn = e & 63; kk = e >> 6; }
      const int gn = n0 + nn, gk = k0 + kk;
      double v = 0.0;
      if (gn < d.N && gk < kmax && !((d.flags & G_TRIB) && gk > gn))
        v = tb ? d.B[gn + (int64_t)gk * d.ldb] : d.B[gk + (int64_t)gn * d.ldb];
      Bs[kk][nn] = T(v);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ty + 16 * q];
        b[q] = Bs[kk][tx + 16 * q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int gm = m0 + ty + 16 * p;
    if (gm >= d.M) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gn = n0 + tx + 16 * q;
      if (gn >= d.N) continue;
      double* c = d.C + gm + (int64_t)gn * d.ldc;
      double v = d.alpha * (double)acc[p][q];
      if (d.beta != 0.0) v += d.beta * (*c);
      *c = v;
    }
  }
}

void launch_gemm(const GemmDesc* d, const TileRef* tiles, int64_t ntiles, int prec, hipStream_t s) {
  if (ntiles == 0) return;
  if (prec == 0)
    hipLaunchKernelGGL(k_gemm<double>, dim3(ntiles), dim3(WG), 0, s, d, tiles);
  else
    hipLaunchKernelGGL(k_gemm<float>, dim3(ntiles), dim3(WG), 0, s, d, tiles);
}

// ---------------------------------------------------------------- Schur reduce
__global__ void __launch_bounds__(WG) k_reduce(const ReduceDesc* __restrict__ descs,
                                               const ContribDesc* __restrict__ cs) {
  const ReduceDesc d = descs[blockIdx.x];
  const int64_t cnt = (int64_t)d.rows * d.cols;
  for (int64_t e = threadIdx.x; e < cnt; e += WG) {
    const int r = (int)(e % d.rows), c = (int)(e / d.rows);
    const bool mirror = d.diag && r < c;
    double sum = 0.0;
    for (int q = d.c_begin; q < d.c_end; ++q) {
      const ContribDesc cd = cs[q];
      sum += mirror ? cd.C[c + (int64_t)r * cd.ldC] : cd.C[r + (int64_t)c * cd.ldC];
    }
    d.T[r + (int64_t)c * d.ldT] -= sum;
  }
}

void launch_reduce(const ReduceDesc* d, int32_t count, const ContribDesc* c, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_reduce, dim3(count), dim3(WG), 0, s, d, c);
}

// ---------------------------------------------------------------- copies
__global__ void __launch_bounds__(WG) k_copy(const CopyDesc* __restrict__ descs) {
  const CopyDesc d = descs[blockIdx.x];
  const int64_t cnt = (int64_t)d.rows * d.cols;
  for (int64_t e = threadIdx.x; e < cnt; e += WG) {
    const int r = (int)(e % d.rows), c = (int)(e / d.rows);
    d.dst[r + (int64_t)c * d.ldd] = d.trans ? d.src[c + (int64_t)r * d.lds] : d.src[r + (int64_t)c * d.lds];
  }
}

void launch_copy(const CopyDesc* d, int64_t count, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_copy, dim3(count), dim3(WG), 0, s, d);
}

__global__ void k_set_identity(double* const* diag, const int32_t* n, const int32_t* ld) {
  double* D = diag[blockIdx.x];
  const int m = n[blockIdx.x], l = ld[blockIdx.x];
  for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += blockDim.x) {
    const int r = (int)(e % m), c = (int)(e / m);
    D[r + (int64_t)c * l] = (r == c) ? 1.0 : 0.0;
  }
}

void launch_set_identity(double* const* diag, const int32_t* n, const int32_t* ld, int32_t count, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_set_identity, dim3(count), dim3(WG), 0, s, diag, n, ld);
}

}  // namespace spand
