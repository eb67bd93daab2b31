// Blocked Cholesky building blocks (Sec. 2.4 pivot blocks, Sec. 2.5 interface
// blocks), run in lockstep over every panel of a level by the host driver:
//
//   for kb = 0, NB, 2NB, ...:
//     k_potrf_diag   factor the w x w diagonal block D = P[kb:kb+w, kb:kb+w] in LDS,
//                    write L_kk back and D_k^{-1} = L_kk^{-1} to the inverse store;
//     k_panel_trsm   P[kb+w:, kb:kb+w] <- P[kb+w:, kb:kb+w] L_kk^{-T} (in place, row per thread);
//     trailing GEMM  P[kb+w:, kb+w:n] -= P[kb+w:, kb:kb+w] P[kb+w:n, kb:kb+w]^T (k_gemm).
//
// Applied to the panel [A_ss; A_{N_s s}] this leaves [L_s; A_{N_s s} L_s^{-T}], i.e. the
// factor and G of the elimination; applied to an interface panel it leaves L_p on
// top and the right-scaled blocks below.  The left scaling by L_i^{-1} of block
// (i, p) is the same recurrence from the left:
//     GEMM (in place, lower-triangular L_kk^{-1})  X[kb:kb+w, :] <- L_kk^{-1} X[kb:kb+w, :]
//     GEMM              X[kb+w:, :] -= L[kb+w:, kb:kb+w] X[kb:kb+w, :]
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace spand {

#define PW 256

// Loads below are issued from addresses clamped into the block, never behind a
// branch, so that a thread's loads are all in flight together; entries read past
// the block are replaced or never used in a stored result.
typedef __attribute__((address_space(1))) const double gdouble_c;
typedef __attribute__((address_space(1))) double gdouble_w;
__device__ inline double gldc(const double* p) { return *(gdouble_c*)p; }
// stores through the global address space do not count against the LDS counter,
// so a later LDS read never waits for them
__device__ inline void gstc(double* p, double v) { *(gdouble_w*)p = v; }

// Xi[r][c] = D[r + c * w] for r, c < w (the entries beyond w are left as they are)
__device__ inline void stage_inverse(const double* __restrict__ D, int w, double (*Xi)[CHOL_NB + 1]) {
  const int r = threadIdx.x & 63, c0 = threadIdx.x >> 6;
  const int rc = r < w ? r : w - 1;
  double v[CHOL_NB / 4];
#pragma unroll
  for (int u = 0; u < CHOL_NB / 4; ++u) {
    const int c = c0 + 4 * u;
    v[u] = gldc(D + rc + (c < w ? c : w - 1) * w);
  }
#pragma unroll
  for (int u = 0; u < CHOL_NB / 4; ++u) {
    const int c = c0 + 4 * u;
    if (r < w && c < w) Xi[r][c] = v[u];
  }
}

// One diagonal block per workgroup.  Cholesky column by column in LDS: thread t
// updates column j = t % 64 of rows t / 64, t / 64 + 4, ... (no index division);
// then lane c of wave 0 forms column c of L^{-1} by forward substitution, entirely
// in registers (the rows of L are broadcast from LDS).
__global__ void __launch_bounds__(PW, 3) k_potrf_diag(const PotrfDesc* __restrict__ descs) {
  const PotrfDesc d = descs[blockIdx.x];
  const int w = d.w;
  __shared__ double D[CHOL_NB][CHOL_NB + 1];
  __shared__ double diag[CHOL_NB];  // L_kk; D[k][k] keeps the pivot, so it is read without a barrier
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int jc = tid & 63, i0 = tid >> 6;  // column and first row of this thread's share
  if (tid == 0) bad = 0;
  if (tid < CHOL_NB) diag[tid] = 1.0;
  {
    const int jcc = jc < w ? jc : w - 1;
    double v[CHOL_NB / 4];
#pragma unroll
    for (int s = 0; s < CHOL_NB / 4; ++s) {
      const int r = i0 + 4 * s;
      v[s] = gldc(d.P + (r < w ? r : w - 1) + (int64_t)jcc * d.ld);
    }
#pragma unroll
    for (int s = 0; s < CHOL_NB / 4; ++s) {
      const int r = i0 + 4 * s;
      D[r][jc] = (r < w && jc < w && r >= jc) ? v[s] : 0.0;
    }
  }
  __syncthreads();
  for (int k = 0; k < w; ++k) {
    double piv = D[k][k];
    if (!(piv > 0.0) || !isfinite(piv)) {
      piv = 1.0;
      if (tid == 0) bad = 1;
    }
    const double rk = sqrt(piv);
    if (tid < 64) {  // nobody reads column k below the diagonal in this phase
      if (tid == k) diag[k] = rk;
      if (tid > k && tid < w) D[tid][k] /= rk;
    }
    __syncthreads();
    if (jc > k && jc < w) {
      const double ljk = D[jc][k];
#pragma unroll
      for (int s = 0; s < CHOL_NB / 4; ++s) {
        const int r = i0 + 4 * s;
        if (r >= jc && r < w) D[r][jc] -= D[r][k] * ljk;
      }
    }
    __syncthreads();
  }
  // L^{-1}: column c, X[i][c] = (delta_ic - sum_{c <= q < i} L[i][q] X[q][c]) / L[i][i]
  if (tid < 64) {
    const int c = tid;
    double x[CHOL_NB];
#pragma unroll
    for (int i = 0; i < CHOL_NB; ++i) {
      double acc = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int q = 0; q < i; ++q) acc = fma(-D[i][q], x[q], acc);
      x[i] = (i >= c && i < w) ? acc / diag[i] : 0.0;
    }
    if (c < w)
#pragma unroll
      for (int i = 0; i < CHOL_NB; ++i)
        if (i < w) gstc(d.Dinv + i + (int64_t)c * w, x[i]);
  }
#pragma unroll
  for (int s = 0; s < CHOL_NB / 4; ++s) {
    const int r = i0 + 4 * s;
    if (r < w && jc < w && r >= jc) gstc(d.P + r + (int64_t)jc * d.ld, r == jc ? diag[jc] : D[r][jc]);
  }
  if (bad && tid == 0) atomicMin(d.fail, d.id);
}

// rows [r0, r1) of the panel below the diagonal block: x <- x L_kk^{-T}, computed as
// the transposed rows Y^T = L_kk^{-1} X^T on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64; lane l holds A[l%16][l/16], B[l/16][l%16], and entry q
// of the result C[l/16 + 4q][l%16]).  Wave v takes rows r0 + 64 v .. + 63: the B
// entries are 16 consecutive rows of one column of the panel, the A entries come
// from the inverse staged in LDS (zero outside w x w; it is zero above its
// diagonal), and the results go back with 16 lanes on 16 consecutive rows.  Every
// row of a wave is read before the wave stores any, so the update is in place.
// Each step adds its four products in k order, as a plain FMA loop would.
typedef double dbl4_c __attribute__((ext_vector_type(4)));
__device__ const double g_chol_zero[1] = {0.0};
__global__ void __launch_bounds__(PW) k_panel_trsm(const PanelDesc* __restrict__ descs) {
  const PanelDesc d = descs[blockIdx.x];
  const int w = d.w;
  __shared__ double Xi[CHOL_NB][CHOL_NB + 1];  // Xi[c][k] = L_kk^{-1}[c][k]
  {
    const int r = threadIdx.x & 63, c0 = threadIdx.x >> 6;
    const int rc = r < w ? r : w - 1;
    double v[CHOL_NB / 4];
#pragma unroll
    for (int u = 0; u < CHOL_NB / 4; ++u) {
      const int c = c0 + 4 * u;
      v[u] = gldc(d.Dinv + rc + (c < w ? c : w - 1) * w);
    }
#pragma unroll
    for (int u = 0; u < CHOL_NB / 4; ++u) {
      const int c = c0 + 4 * u;
      Xi[r][c] = (r < w && c < w) ? v[u] : 0.0;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
  const int rb0 = d.r0 + 64 * (threadIdx.x >> 6);
  if (rb0 >= d.r1) return;  // no barrier follows
  dbl4_c acc[4][4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[cb][rb] = dbl4_c{0.0, 0.0, 0.0, 0.0};
  // entries past r1 or w read a zero constant
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    double b[8][4];
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const int r = rb0 + 16 * rb + i, k = 4 * (8 * h + j) + kq;
        const bool ok = r < d.r1 && k < w;
        b[j][rb] = gldc(ok ? d.P + r + (int64_t)k * d.ld : g_chol_zero);
      }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 4 * (8 * h + j) + kq;
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const double a = Xi[16 * cb + i][k];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) acc[cb][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[j][rb], acc[cb][rb], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int r = rb0 + 16 * rb + i;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = 16 * cb + kq + 4 * q;
        if (r < d.r1 && c < w) gstc(d.P + r + (int64_t)c * d.ld, acc[cb][rb][q]);
      }
    }
}

void launch_potrf_diag(const PotrfDesc* d, int32_t count, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_potrf_diag, dim3(count), dim3(PW), 0, s, d);
}
void launch_panel_trsm(const PanelDesc* d, int32_t count, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_panel_trsm, dim3(count), dim3(PW), 0, s, d);
}

}  // namespace spand
