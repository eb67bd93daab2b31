// Interpolative sparsification (Sec. 2.6.2) on the GPU: the pieces around the
// truncated CPQR of A_np, and the preconditioner apply of such an interface.
//
// For an interface p of np dofs with r coarse dofs c = perm[0..r) (the CPQR pivots
// in pivot order) and nf = np - r fine dofs f = perm[r..np):
//   k_interp_perm   perm from the pivots
//   k_interp_t      T_cf = R_11^{-1} R_12 by back substitution (one wave per column)
//   k_interp_x      X = A_pp in (f, c) order, symmetric, from A_pp's lower triangle
//   k_interp_rows   the rows c of every block A_pq, from a copy of A_np
// The congruence products, the Cholesky of C_ff and the update of A_cc run on the
// batched GEMM and blocked Cholesky of the elimination.
//
// The apply of one interface (one wave per interface and right-hand side, the
// interface's values in LDS):
//   forward   y_f = L_f^{-1} (x_f - T^T x_c),  y_c = x_c - G y_f
//   backward  y_f = L_f^{-T} (y_f - G^T y_c),  x_c = y_c - T y_f,  x_f = y_f
#include <hip/hip_runtime.h>

#include "apply.h"
#include "kernels.h"

namespace spand {

namespace {

__device__ inline double isum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace

__global__ void __launch_bounds__(256) k_interp_perm(const InterpPermDesc* __restrict__ ds) {
  const InterpPermDesc d = ds[blockIdx.x];
  __shared__ unsigned char mark[INTERP_MAX_NP];
  __shared__ int wtot[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = tid; j < d.np; j += 256) mark[j] = 0;
  __syncthreads();
  for (int i = tid; i < d.r; i += 256) {
    const int c = min(max(d.piv[i], 0), d.np - 1);
    mark[c] = 1;
    d.perm[i] = c;
  }
  __syncthreads();
  int run = 0;
  for (int c0 = 0; c0 < d.np; c0 += 256) {
    const int j = c0 + tid;
    const bool fine = j < d.np && mark[j] == 0;
    const unsigned long long bal = __ballot(fine);
    const int below = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wtot[wave] = __popcll(bal);
    __syncthreads();
    int off = run;
    for (int w = 0; w < wave; ++w) off += wtot[w];
    if (fine && d.r + off + below < d.np) d.perm[d.r + off + below] = j;
    run += wtot[0] + wtot[1] + wtot[2] + wtot[3];
    __syncthreads();
  }
}

// One wave per column j of T: x = R_12[:, j], then R_11 x = that column, from the last
// row up (column-oriented: x_k = x_k / R_kk, then x_i -= R_ik x_k for i < k).
__global__ void __launch_bounds__(64) k_interp_t(const InterpTDesc* __restrict__ ds,
                                                 const InterpCol* __restrict__ cols) {
  extern __shared__ double xs[];
  const InterpCol c = cols[blockIdx.x];
  const InterpTDesc d = ds[c.desc];
  const int lane = threadIdx.x, r = d.r;
  const double* R12 = d.W + (int64_t)d.perm[r + c.j] * d.ldw;
  for (int i = lane; i < r; i += 64) xs[i] = R12[i];
  __syncthreads();
  for (int k = r - 1; k >= 0; --k) {
    const double* Rk = d.W + (int64_t)d.perm[k] * d.ldw;
    const double xk = xs[k] / Rk[k];
    __syncthreads();
    if (lane == 0) xs[k] = xk;
    for (int i = lane; i < k; i += 64) xs[i] -= Rk[i] * xk;
    __syncthreads();
  }
  double* out = d.T + (int64_t)c.j * r;
  for (int i = lane; i < r; i += 64) out[i] = xs[i];
}

__global__ void __launch_bounds__(256) k_interp_x(const InterpXDesc* __restrict__ ds) {
  const InterpXDesc d = ds[blockIdx.x];
  const int nf = d.np - d.r;
  for (int64_t e = d.e0 + threadIdx.x; e < d.e1; e += 256) {
    const int a = (int)(e % d.np), b = (int)(e / d.np);
    const int i = d.perm[a < nf ? d.r + a : a - nf];
    const int j = d.perm[b < nf ? d.r + b : b - nf];
    d.X[e] = (i >= j) ? d.App[i + (int64_t)j * d.lda] : d.App[j + (int64_t)i * d.lda];
  }
}

__global__ void __launch_bounds__(256) k_interp_rows(const InterpRowDesc* __restrict__ ds) {
  const InterpRowDesc d = ds[blockIdx.x];
  for (int64_t e = d.e0 + threadIdx.x; e < d.e1; e += 256) {
    const int i = (int)(e % d.r), k = (int)(e / d.r);
    const double v = d.keep[d.row0 + k + (int64_t)d.perm[i] * d.ldk];
    if (d.trans)
      d.blk[k + (int64_t)i * d.ld] = v;
    else
      d.blk[i + (int64_t)k * d.ld] = v;
  }
}

void launch_interp_perm(const InterpPermDesc* d, int32_t count, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_interp_perm, dim3(count), dim3(256), 0, s, d);
}

void launch_interp_t(const InterpTDesc* d, const InterpCol* cols, int64_t ncols, int32_t rmax, hipStream_t s) {
  if (ncols > 0)
    hipLaunchKernelGGL(k_interp_t, dim3(unsigned(ncols)), dim3(64), size_t(rmax > 0 ? rmax : 1) * sizeof(double), s, d,
                       cols);
}

void launch_interp_x(const InterpXDesc* d, int64_t count, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_interp_x, dim3(unsigned(count)), dim3(256), 0, s, d);
}

void launch_interp_rows(const InterpRowDesc* d, int64_t count, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_interp_rows, dim3(unsigned(count)), dim3(256), 0, s, d);
}

// ---------------------------------------------------------------- apply
// Interface blockIdx.x, right-hand side blockIdx.y; one wave.  y holds the np values
// of the interface in (c, f) order.
template <int DIR>
__global__ void __launch_bounds__(64) k_interp_apply(const InterpAp* __restrict__ ds, ApplyArgs a) {
  __shared__ double y[INTERP_MAX_NP];
  const InterpAp d = ds[blockIdx.x];
  const int lane = threadIdx.x, np = d.np, r = d.r, nf = np - r;
  double* x = a.x + (int64_t)blockIdx.y * a.ldx;
  const int32_t* sl = a.slot + d.slot_p;
  const double* T = d.T;
  const double* L = d.X;       // L_f: rows and columns 0..nf
  const double* G = d.X + nf;  // G_cf: rows nf..np, columns 0..nf
  const int64_t ld = np;
  if (DIR > 0) {
    for (int e = lane; e < np; e += 64) y[e] = x[sl[d.perm[e]]];
    __syncthreads();
    // y_f -= T^T y_c
    for (int j = 0; j < nf; ++j) {
      double s = 0.0;
      for (int i = lane; i < r; i += 64) s = fma(T[i + (int64_t)j * r], y[i], s);
      s = isum(s);
      if (lane == 0) y[r + j] -= s;
    }
    __syncthreads();
    // y_f <- L_f^{-1} y_f
    for (int k = 0; k < nf; ++k) {
      const double yk = y[r + k] / L[k + k * ld];
      __syncthreads();
      if (lane == 0) y[r + k] = yk;
      for (int i = k + 1 + lane; i < nf; i += 64) y[r + i] -= L[i + k * ld] * yk;
      __syncthreads();
    }
    // y_c -= G y_f
    for (int i = lane; i < r; i += 64) {
      double s = 0.0;
      for (int j = 0; j < nf; ++j) s = fma(G[i + j * ld], y[r + j], s);
      y[i] -= s;
    }
    __syncthreads();
    for (int e = lane; e < np; e += 64) x[sl[e]] = y[e];
  } else {
    for (int e = lane; e < np; e += 64) y[e] = x[sl[e]];
    __syncthreads();
    // y_f -= G^T y_c
    for (int j = 0; j < nf; ++j) {
      double s = 0.0;
      for (int i = lane; i < r; i += 64) s = fma(G[i + j * ld], y[i], s);
      s = isum(s);
      if (lane == 0) y[r + j] -= s;
    }
    __syncthreads();
    // y_f <- L_f^{-T} y_f, from the last row up
    for (int k = nf - 1; k >= 0; --k) {
      double s = 0.0;
      for (int i = k + 1 + lane; i < nf; i += 64) s = fma(L[i + k * ld], y[r + i], s);
      s = isum(s);
      const double yk = (y[r + k] - s) / L[k + k * ld];
      __syncthreads();
      if (lane == 0) y[r + k] = yk;
      __syncthreads();
    }
    // x_c = y_c - T y_f
    for (int i = lane; i < r; i += 64) {
      double s = 0.0;
      for (int j = 0; j < nf; ++j) s = fma(T[i + (int64_t)j * r], y[r + j], s);
      y[i] -= s;
    }
    __syncthreads();
    for (int e = lane; e < np; e += 64) x[sl[d.perm[e]]] = y[e];
  }
}

void launch_interp_apply(const InterpAp* d, int32_t count, const ApplyArgs& a, int dir, hipStream_t s) {
  if (count <= 0) return;
  if (dir > 0)
    hipLaunchKernelGGL(k_interp_apply<1>, dim3(count, a.nrhs), dim3(64), 0, s, d, a);
  else
    hipLaunchKernelGGL(k_interp_apply<-1>, dim3(count, a.nrhs), dim3(64), 0, s, d, a);
}

}  // namespace spand
