// Preconditioner apply z = F^T F r (F = M^T, Sec. 2.8) and the FP64 PCG vector
// kernels.  Vectors are n x nrhs column-major (FP64); the dofs of a cluster are
// addressed through its slot list (vertex ids of the dofs it currently carries).
//
// Forward sweep of one step (levels L -> 1):
//   k_elim_fwd    x_s <- L_s^{-1} x_s            (one workgroup per eliminated s;
//                                                  blocked substitution with the
//                                                  inverses of the diagonal blocks)
//   k_fwd_gemv    y_s <- G_{N_s s} x_s            (one workgroup per 64 panel rows of
//                                                  s, on the panel's 128-byte lines)
//   k_target_sum  x_n <- x_n - sum_s y_s (rows of n) (contributions in ascending s)
//   k_iface<1>    x_p <- Q_p^T L_p^{-1} x_p      (interfaces of at most 128 dofs, one wave each)
//   k_scale<1>    x_p <- L_p^{-1} x_p                (larger interfaces: explicit inverse, 64-row tiles)
//   k_house_*     x_p <- Q_p^T x_p                (compact WY form, three tile launches)
//   k_interp_apply<1>  interpolative interfaces (Sec. 2.6.2, kernels_interp.hip)
// Backward sweep (levels 1 -> L), the transposes in reverse order:
//   k_interp_apply<-1>
//   k_iface<-1>   x_p <- L_p^{-T} Q_p x_p
//   k_house_*     x_p <- Q_p x_p
//   k_scale<-1>   x_p <- L_p^{-T} x_p
//   k_gather         neighbour dofs of every s into a contiguous buffer
//   k_elim_bwd_gemv  t_s <- x_s - G_{N_s s}^T x_{N_s}  (one workgroup per 64 columns of s)
//   k_elim_bwd       x_s <- L_s^{-T} t_s
#include <hip/hip_runtime.h>

#include "apply.h"
#include "kernels.h"

namespace spand {

#define AW 256
#define RB 8  // right-hand sides per register pass

__device__ inline double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------- tile GEMVs
// The products of a 64 x 64 tile of a factor block with a 64 x RB block of
// right-hand sides run on the FP64 matrix cores (v_mfma_f64_16x16x4f64: C 16x16 +=
// A 16x4 B 4x16; lane l holds A[l%16][l/16] and B[l/16][l%16], and entry q of the
// result C[l/16 + 4q][l%16]).  Wave w owns output rows (or columns) 16w..16w+15 of
// the tile over all of k, so its sums need no combining with the other waves; the
// RB right-hand sides fill half of the 16 B columns, the other half is zero.  Each
// step adds its four products to the accumulator in k order, as a plain FMA loop
// would.  The x tile is staged in LDS (double buffered, one barrier per tile) and
// two tiles are in flight: tile t + 2 is requested into the registers that tile t
// has just left.  Matrix entries are read with buffer loads: a 32-bit offset per
// entry from a descriptor of the block; an entry outside the matrix gets an offset
// past the descriptor's range and reads as zero, so no loaded value is consumed
// before its use.  Vector entries outside x read a zero constant instead.
typedef double dbl4 __attribute__((ext_vector_type(4)));
static_assert(RB == 8, "the MFMA tiles fill 8 of the 16 B columns");
__device__ const double g_zero[1] = {0.0};

struct TileShared {
  double A[64][65];     // staged tile of the transposed product
  double x[2][64][RB];  // x tiles
  double out[64][RB];   // results handed to the row-per-thread layout
};

typedef __attribute__((address_space(1))) const double gdouble;
__device__ inline double gld(const double* p) { return *(gdouble*)p; }

// Descriptor of the entries [0, n) of a block (n * 8 < 2^31 bytes for the factor
// blocks), and entry e of it, or zero when !ok.
__device__ inline __amdgpu_buffer_rsrc_t block_rsrc(const double* A, int64_t n) {
  const int64_t bytes = n * 8 < 0x7FFFFFF0LL ? n * 8 : 0x7FFFFFF0LL;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(A), 0, (int)bytes, 0x00020000);
}
__device__ inline double bld(__amdgpu_buffer_rsrc_t r, unsigned e, bool ok) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, ok ? e * 8u : 0x80000000u, 0, 0));
}

// x rows k0 + lane of the RB right-hand sides owned by this thread: x[k] or, with a
// slot list, x[xsl[k]]
__device__ inline void xtile_load(const double* __restrict__ x, int64_t ldx, int k0, int nk, int nr,
                                  const int32_t* __restrict__ xsl, double (&xv)[2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool kok = k0 + lane < nk;
  const int64_t xr = kok ? (xsl ? (int64_t)xsl[k0 + lane] : (int64_t)(k0 + lane)) : 0;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int c = w + 4 * u;
    xv[u] = gld(kok && c < nr ? x + xr + (int64_t)c * ldx : g_zero);
  }
}
__device__ inline void xtile_store(const double (&xv)[2], double (*xs)[RB]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  xs[lane][w] = xv[0];
  xs[lane][w + 4] = xv[1];
}
// 16 MFMA steps over a 64-deep k tile; av[j] is this lane's A entry of step j, the
// B entries come from the k x RB block xs
__device__ inline void mfma_tile(const double (&av)[16], const double (*xs)[RB], dbl4& c) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const double bv = xs[4 * j + kq][i & 7];
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j], i < RB ? bv : 0.0, c, 0, 0, 0);
  }
}
// acc[0], acc[1] += rows (lane, w) and (lane, w + 4) of the 64 x RB result c of the waves
__device__ inline void mfma_out(const dbl4& c, TileShared& sh, double acc[2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, i = lane & 15, kq = lane >> 4;
  if (i < RB) {
#pragma unroll
    for (int q = 0; q < 4; ++q) sh.out[16 * w + kq + 4 * q][i] = c[q];
  }
  __syncthreads();
  acc[0] += sh.out[lane][w];
  acc[1] += sh.out[lane][w + 4];
  __syncthreads();
}

// c += A[r0 + 16 wave + .., k] x[k], k < ncols (rows beyond nrows read as zero), in
// the MFMA layout.  The A entries go straight into registers: the 16 lanes of a step
// read 16 consecutive rows of one column.  tpar counts the x tiles staged so far, so
// that consecutive calls keep alternating the two x buffers.
__device__ void mfma_n_acc(const double* __restrict__ A, int ld, int r0, int nrows, int ncols,
                           const double* __restrict__ x, int64_t ldx, int nr, TileShared& sh, dbl4& c, int& tpar,
                           const int32_t* __restrict__ xsl = nullptr, int rlo = 0) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, i = lane & 15, kq = lane >> 4;
  const int row = r0 + 16 * w + i;
  const bool rok = row >= rlo && row < nrows;
  const int nt = (ncols + 63) >> 6;
  const __amdgpu_buffer_rsrc_t ar = block_rsrc(A, ncols > 0 ? (int64_t)(ncols - 1) * ld + nrows : 0);
  double a0[16], a1[16], x0[2], x1[2];
  auto load = [&](int t, double (&a)[16], double (&xv)[2]) {
    const int k0 = 64 * t;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int k = k0 + 4 * j + kq;
      a[j] = bld(ar, (unsigned)row + (unsigned)k * (unsigned)ld, rok && k < ncols);
    }
    xtile_load(x, ldx, k0, ncols, nr, xsl, xv);
  };
  auto use = [&](int t, const double (&a)[16], const double (&xv)[2]) {
    const int b = (tpar + t) & 1;
    xtile_store(xv, sh.x[b]);
    __syncthreads();
    mfma_tile(a, sh.x[b], c);
  };
  if (nt > 0) load(0, a0, x0);
  if (nt > 1) load(1, a1, x1);
  for (int t = 0; t < nt; t += 2) {
    use(t, a0, x0);
    if (t + 2 < nt) load(t + 2, a0, x0);
    if (t + 1 < nt) {
      use(t + 1, a1, x1);
      if (t + 3 < nt) load(t + 3, a1, x1);
    }
  }
  tpar += nt;
}

// acc += A[(r0 + rr) + k*ld] x[k], k < ncols (rows below rlo or from nrows on read as zero)
__device__ void tile_gemv_n(const double* __restrict__ A, int ld, int r0, int nrows, int ncols,
                            const double* __restrict__ x, int64_t ldx, int nr, TileShared& sh, double acc[2],
                            const int32_t* __restrict__ xsl = nullptr, int rlo = 0) {
  dbl4 c = {0.0, 0.0, 0.0, 0.0};
  int tpar = 0;
  mfma_n_acc(A, ld, r0, nrows, ncols, x, ldx, nr, sh, c, tpar, xsl, rlo);
  __syncthreads();  // the last x tile has been read
  mfma_out(c, sh, acc);
}

// acc += sum_{r < nrows} A[r + (c0 + cc)*ld] x[r] for columns c0 + cc < ncols.  The
// tile is read with lanes down a column and staged in LDS; the MFMA steps read it
// across columns.
__device__ void tile_gemv_t(const double* __restrict__ A, int ld, int c0, int ncols, int nrows,
                            const double* __restrict__ x, int64_t ldx, int nr, TileShared& sh, double acc[2],
                            const int32_t* __restrict__ xsl = nullptr) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, i = lane & 15, kq = lane >> 4;
  const int nt = (nrows + 63) >> 6;
  const __amdgpu_buffer_rsrc_t ar = block_rsrc(A, nrows > 0 ? (int64_t)(ncols - 1) * ld + nrows : 0);
  dbl4 c = {0.0, 0.0, 0.0, 0.0};
  double a0[16], a1[16], x0[2], x1[2];
  auto load = [&](int t, double (&a)[16], double (&xv)[2]) {
    const int k0 = 64 * t;
    const bool rok = k0 + lane < nrows;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int col = c0 + w + 4 * u;
      a[u] = bld(ar, (unsigned)(k0 + lane) + (unsigned)col * (unsigned)ld, rok && col < ncols);
    }
    xtile_load(x, ldx, k0, nrows, nr, xsl, xv);
  };
  auto use = [&](int t, const double (&a)[16], const double (&xv)[2]) {
    __syncthreads();  // the previous tile's A has been read
#pragma unroll
    for (int u = 0; u < 16; ++u) sh.A[lane][w + 4 * u] = a[u];
    xtile_store(xv, sh.x[t & 1]);
    __syncthreads();
    double av[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) av[j] = sh.A[4 * j + kq][16 * w + i];
    mfma_tile(av, sh.x[t & 1], c);
  };
  if (nt > 0) load(0, a0, x0);
  if (nt > 1) load(1, a1, x1);
  for (int t = 0; t < nt; t += 2) {
    use(t, a0, x0);
    if (t + 2 < nt) load(t + 2, a0, x0);
    if (t + 1 < nt) {
      use(t + 1, a1, x1);
      if (t + 3 < nt) load(t + 3, a1, x1);
    }
  }
  __syncthreads();
  mfma_out(c, sh, acc);
}

// ---------------------------------------------------------------- triangular solves
// Blocked solves on a vector segment v (n rows, nr <= RB columns, ld ldv) in the
// apply scratch.  L is lower triangular (ld); its CHOL_NB-wide diagonal blocks have
// the inverses Dinv (block k at k*CHOL_NB^2, ld = block width).  The product with a
// diagonal block runs on the matrix cores like the tiles above; its entries are
// requested before the block's off-diagonal product so that the two loads overlap.
static_assert(CHOL_NB == 64, "tile solves assume 64-wide diagonal blocks");

// this lane's MFMA entries of D (w x w, ld w, zero outside): D[16 wave + l%16][4 j + l/16],
// or of D^T when TR
template <bool TR>
__device__ inline void load_dinv(const double* __restrict__ D, int wd, double (&d)[16]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, i = lane & 15, kq = lane >> 4;
  const int o = 16 * w + i;
  const __amdgpu_buffer_rsrc_t dr = block_rsrc(D, (int64_t)wd * wd);
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int k = 4 * j + kq;
    d[j] = bld(dr, TR ? (unsigned)(k + o * wd) : (unsigned)(o + k * wd), o < wd && k < wd);
  }
}
// v[kb + row] (row < wd) <- the rows of D sh.out (or D^T sh.out) held by this lane
__device__ inline void dinv_apply(const double (&d)[16], TileShared& sh, int wd, double* v, int64_t ldv, int nr) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, i = lane & 15, kq = lane >> 4;
  dbl4 c = {0.0, 0.0, 0.0, 0.0};
  mfma_tile(d, sh.out, c);
  if (i < nr) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = 16 * w + kq + 4 * q;
      if (row < wd) v[row + (int64_t)i * ldv] = c[q];
    }
  }
}

// L y = v in place: y_k = D_k^{-1} (v_k - L[k, :k] y[:k])
__device__ void trsv_fwd(const double* __restrict__ L, int ld, const double* __restrict__ Dinv, int n, double* v,
                         int64_t ldv, int nr, TileShared& sh) {
  const int rr = threadIdx.x & 63, g = threadIdx.x >> 6;
  for (int kb = 0; kb < n; kb += 64) {
    const int w = min(64, n - kb);
    double d[16];
    load_dinv<false>(Dinv + (int64_t)(kb / 64) * 64 * 64, w, d);
    double acc[2] = {0.0, 0.0};
    tile_gemv_n(L + kb, ld, 0, w, kb, v, ldv, nr, sh, acc);
    if (rr < w) {
      sh.out[rr][g] = (g < nr ? v[kb + rr + (int64_t)g * ldv] : 0.0) - acc[0];
      sh.out[rr][g + 4] = (g + 4 < nr ? v[kb + rr + (int64_t)(g + 4) * ldv] : 0.0) - acc[1];
    } else {
      sh.out[rr][g] = 0.0;
      sh.out[rr][g + 4] = 0.0;
    }
    __syncthreads();
    dinv_apply(d, sh, w, v + kb, ldv, nr);
    __threadfence_block();
    __syncthreads();
  }
}

// L^T x = v in place: x_k = D_k^{-T} (v_k - L[k+1:, k]^T x[k+1:])
__device__ void trsv_bwd(const double* __restrict__ L, int ld, const double* __restrict__ Dinv, int n, double* v,
                         int64_t ldv, int nr, TileShared& sh) {
  const int cc = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int nblk = (n + 63) / 64;
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int kb = bi * 64;
    const int w = min(64, n - kb);
    double d[16];
    load_dinv<true>(Dinv + (int64_t)bi * 64 * 64, w, d);
    double acc[2] = {0.0, 0.0};
    tile_gemv_t(L + kb + w, ld, kb, kb + w, n - kb - w, v + kb + w, ldv, nr, sh, acc);
    if (cc < w) {
      sh.out[cc][g] = (g < nr ? v[kb + cc + (int64_t)g * ldv] : 0.0) - acc[0];
      sh.out[cc][g + 4] = (g + 4 < nr ? v[kb + cc + (int64_t)(g + 4) * ldv] : 0.0) - acc[1];
    } else {
      sh.out[cc][g] = 0.0;
      sh.out[cc][g + 4] = 0.0;
    }
    __syncthreads();
    dinv_apply(d, sh, w, v + kb, ldv, nr);
    __threadfence_block();
    __syncthreads();
  }
}

// Row moves between x (through the slots) and the scratch.  The source and the
// destination may alias as far as the compiler knows, so every load of a pass is
// written before its stores; otherwise each load would wait for the store before it.
#define MV_ROWS 4  // rows per thread and pass
template <bool TO_TMP>
__device__ inline void move_seg(const int32_t* sl, int n, const ApplyArgs& a, int64_t off) {
  for (int rb = 0; rb < n; rb += AW * MV_ROWS) {
    int64_t xo[MV_ROWS];
#pragma unroll
    for (int u = 0; u < MV_ROWS; ++u) {  // every slot load issued: rows past n read slot n - 1
      const int r = rb + threadIdx.x + u * AW;
      const int64_t v = sl[r < n ? r : n - 1];
      xo[u] = r < n ? v : -1;
    }
    for (int c0 = 0; c0 < a.nrhs; c0 += RB) {
      double b[MV_ROWS][RB];
#pragma unroll
      for (int u = 0; u < MV_ROWS; ++u) {
        const int64_t to = off + rb + threadIdx.x + u * AW;
#pragma unroll
        for (int c = 0; c < RB; ++c) {
          const bool ok = xo[u] >= 0 && c0 + c < a.nrhs;
          b[u][c] = ok ? (TO_TMP ? a.x[xo[u] + (int64_t)(c0 + c) * a.ldx] : a.tmp[to + (int64_t)(c0 + c) * a.ldt]) : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < MV_ROWS; ++u) {
        const int64_t to = off + rb + threadIdx.x + u * AW;
#pragma unroll
        for (int c = 0; c < RB; ++c)
          if (xo[u] >= 0 && c0 + c < a.nrhs) {
            if (TO_TMP)
              a.tmp[to + (int64_t)(c0 + c) * a.ldt] = b[u][c];
            else
              a.x[xo[u] + (int64_t)(c0 + c) * a.ldx] = b[u][c];
          }
      }
    }
  }
}
__device__ inline void gather_seg(const int32_t* sl, int n, const ApplyArgs& a, int64_t off) {
  move_seg<true>(sl, n, a, off);
  __threadfence_block();
  __syncthreads();
}
__device__ inline void scatter_seg(const int32_t* sl, int n, const ApplyArgs& a, int64_t off) {
  move_seg<false>(sl, n, a, off);
}

// ---------------------------------------------------------------- sweep kernels
// y_s = L_s^{-1} x_s; y_s stays in the scratch for the target updates and replaces x_s.
__global__ void __launch_bounds__(AW, 2) k_elim_fwd(const ElimAp* __restrict__ ds, ApplyArgs a) {
  __shared__ TileShared sh;
  const ElimAp e = ds[blockIdx.x];
  const int32_t* sl = a.slot + e.slot_s;
  gather_seg(sl, e.ns, a, e.tmp);
  for (int c0 = 0; c0 < a.nrhs; c0 += RB)
    trsv_fwd(e.L, e.ld, e.Dinv, e.ns, a.tmp + e.tmp + (int64_t)c0 * a.ldt, a.ldt, min(RB, a.nrhs - c0), sh);
  scatter_seg(sl, e.ns, a, e.tmp);
}

// y_s = G_s L_s^{-1} x_s for the panel rows [r0, r0 + 64) of s (those of G: rows ns
// to ns + nN): the tiles follow the panel's 128-byte lines, so every G entry is read
// once, in whole lines; L_s^{-1} x_s comes from the scratch where k_elim_fwd left it.
__global__ void __launch_bounds__(AW) k_fwd_gemv(const ElimAp* __restrict__ ds, const FwdTile* __restrict__ ft,
                                                 ApplyArgs a) {
  __shared__ TileShared sh;
  const FwdTile f = ft[blockIdx.x];
  const ElimAp e = ds[f.s];
  const int rr = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int row = f.r0 + rr;
  const bool rok = row >= e.ns && row < e.ns + e.nN;
  for (int c0 = 0; c0 < a.nrhs; c0 += RB) {
    const int nr = min(RB, a.nrhs - c0);
    double acc[2] = {0.0, 0.0};
    tile_gemv_n(e.L, e.ld, f.r0, e.ns + e.nN, e.ns, a.tmp + e.tmp + (int64_t)c0 * a.ldt, a.ldt, nr, sh, acc,
                nullptr, e.ns);
    if (rok) {
      double* yp = a.tmp + e.ytmp + (row - e.ns) + (int64_t)c0 * a.ldt;
      if (g < nr) yp[(int64_t)g * a.ldt] = acc[0];
      if (g + 4 < nr) yp[(int64_t)(g + 4) * a.ldt] = acc[1];
    }
  }
}

// x_n -= sum_s y_s (the rows of n), the contributions of n in ascending s
__global__ void __launch_bounds__(AW) k_target_sum(const TargetAp* __restrict__ ts, const TargetContrib* __restrict__ cs,
                                                   ApplyArgs a) {
  const TargetAp t = ts[blockIdx.x];
  const int rr = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int r = t.r0 + rr;
  if (r >= t.nn) return;
  const int64_t xo = a.slot[t.slot_n + r];
  for (int c = g; c < a.nrhs; c += 4) {
    double acc = 0.0;
    for (int q = t.cbeg; q < t.cend; ++q) acc += a.tmp[cs[q].y + r + (int64_t)c * a.ldt];
    a.x[xo + (int64_t)c * a.ldx] -= acc;
  }
}

// x_p <- L_p^{-1} x_p (DIR = +1) or L_p^{-T} x_p (DIR = -1) with the explicit inverse:
// x_p is gathered into the scratch first (k_gather_rows), then one workgroup per
// 64 rows writes its rows of the product back through the slots.
__global__ void k_gather_rows(const int32_t* __restrict__ sg, int64_t len, ApplyArgs a) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= len) return;
  const int32_t v = sg[t];
  for (int c0 = 0; c0 < a.nrhs; c0 += RB) {
    double b[RB];
#pragma unroll
    for (int c = 0; c < RB; ++c) b[c] = c0 + c < a.nrhs ? a.x[v + (int64_t)(c0 + c) * a.ldx] : 0.0;
#pragma unroll
    for (int c = 0; c < RB; ++c)
      if (c0 + c < a.nrhs) a.tmp[t + (int64_t)(c0 + c) * a.ldt] = b[c];
  }
}

template <int DIR>
__global__ void __launch_bounds__(AW) k_scale(const ScaleAp* __restrict__ ds, const ScaleTile* __restrict__ tl,
                                              ApplyArgs a) {
  __shared__ TileShared sh;
  const ScaleTile st = tl[blockIdx.x];
  const ScaleAp e = ds[st.p];
  const int np = e.np, r0 = st.r0;
  const int32_t* sl = a.slot + e.slot_p;
  const int rr = threadIdx.x & 63, g = threadIdx.x >> 6;
  const double* xs = a.tmp + e.tmp;
  for (int c0 = 0; c0 < a.nrhs; c0 += RB) {
    const int nr = min(RB, a.nrhs - c0);
    const int64_t co = (int64_t)c0 * a.ldt;
    double acc[2] = {0.0, 0.0};
    if (DIR > 0)  // rows r0.. of L^{-1} x: columns up to the diagonal tile
      tile_gemv_n(e.Linv, e.ldl, r0, np, min(np, r0 + 64), xs + co, a.ldt, nr, sh, acc);
    else          // rows r0.. of L^{-T} x: rows r0.. of L^{-1}
      tile_gemv_t(e.Linv + r0, e.ldl, r0, np, np - r0, xs + co + r0, a.ldt, nr, sh, acc);
    if (r0 + rr < np) {
      double* xp = a.x + sl[r0 + rr] + (int64_t)c0 * a.ldx;
      if (g < nr) xp[(int64_t)g * a.ldx] = acc[0];
      if (g + 4 < nr) xp[(int64_t)(g + 4) * a.ldx] = acc[1];
    }
  }
}

// Q_p in compact WY form, Q = I - V T V^T (T upper triangular r x r).  DIR = +1
// applies Q^T = I - V T^T V^T, DIR = -1 applies Q, in three launches over 64-wide
// tiles (scratch of p: [w: r][u: r] per right-hand side):
//   k_house_w    w = V^T x_p           one workgroup per 64 reflectors (x_p read through its slots)
//   k_house_t    u = T^T w or u = T w  one workgroup per 64 reflectors
//   k_house_v    x_p -= V u            one workgroup per 64 rows of p
__global__ void __launch_bounds__(AW) k_house_w(const HouseAp* __restrict__ ds, const HouseTile* __restrict__ tl,
                                                ApplyArgs a) {
  __shared__ TileShared sh;
  const HouseTile ht = tl[blockIdx.x];
  const HouseAp e = ds[ht.p];
  const int np = e.np, r = e.r, j0 = ht.j0;
  const int32_t* sl = a.slot + e.slot_p;
  const int cc = threadIdx.x & 63, g = threadIdx.x >> 6;
  double* ws = a.tmp + e.tmp;
  for (int c0 = 0; c0 < a.nrhs; c0 += RB) {
    const int nr = min(RB, a.nrhs - c0);
    double acc[2] = {0.0, 0.0};
    tile_gemv_t(e.V, e.ldv, j0, r, np, a.x + (int64_t)c0 * a.ldx, a.ldx, nr, sh, acc, sl);
    if (j0 + cc < r) {
      if (g < nr) ws[j0 + cc + (int64_t)(c0 + g) * a.ldt] = acc[0];
      if (g + 4 < nr) ws[j0 + cc + (int64_t)(c0 + g + 4) * a.ldt] = acc[1];
    }
  }
}

template <int DIR>
__global__ void __launch_bounds__(AW) k_house_t(const HouseAp* __restrict__ ds, const HouseTile* __restrict__ tl,
                                                ApplyArgs a) {
  __shared__ TileShared sh;
  const HouseTile ht = tl[blockIdx.x];
  const HouseAp e = ds[ht.p];
  const int r = e.r, j0 = ht.j0;
  const int cc = threadIdx.x & 63, g = threadIdx.x >> 6;
  const double* ws = a.tmp + e.tmp;
  double* us = a.tmp + e.tmp + r;
  for (int c0 = 0; c0 < a.nrhs; c0 += RB) {
    const int nr = min(RB, a.nrhs - c0);
    const int64_t co = (int64_t)c0 * a.ldt;
    double acc[2] = {0.0, 0.0};
    if (DIR > 0)
      tile_gemv_t(e.T, e.ldt, j0, r, r, ws + co, a.ldt, nr, sh, acc);
    else
      tile_gemv_n(e.T, e.ldt, j0, r, r, ws + co, a.ldt, nr, sh, acc);
    if (j0 + cc < r) {
      if (g < nr) us[co + j0 + cc + (int64_t)g * a.ldt] = acc[0];
      if (g + 4 < nr) us[co + j0 + cc + (int64_t)(g + 4) * a.ldt] = acc[1];
    }
  }
}

__global__ void __launch_bounds__(AW) k_house_v(const HouseAp* __restrict__ ds, const HouseTile* __restrict__ tl,
                                                ApplyArgs a) {
  __shared__ TileShared sh;
  const HouseTile ht = tl[blockIdx.x];
  const HouseAp e = ds[ht.p];
  const int np = e.np, r = e.r, r0 = ht.j0;
  const int32_t* sl = a.slot + e.slot_p;
  const int rr = threadIdx.x & 63, g = threadIdx.x >> 6;
  const double* us = a.tmp + e.tmp + r;
  for (int c0 = 0; c0 < a.nrhs; c0 += RB) {
    const int nr = min(RB, a.nrhs - c0);
    double acc[2] = {0.0, 0.0};
    tile_gemv_n(e.V, e.ldv, r0, np, r, us + (int64_t)c0 * a.ldt, a.ldt, nr, sh, acc);
    if (r0 + rr < np) {
      double* xp = a.x + sl[r0 + rr] + (int64_t)c0 * a.ldx;
      const double x0 = g < nr ? xp[(int64_t)g * a.ldx] : 0.0;
      const double x1 = g + 4 < nr ? xp[(int64_t)(g + 4) * a.ldx] : 0.0;
      if (g < nr) xp[(int64_t)g * a.ldx] = x0 - acc[0];
      if (g + 4 < nr) xp[(int64_t)(g + 4) * a.ldx] = x1 - acc[1];
    }
  }
}

// ---------------------------------------------------------------- small interfaces
// One wave per interface p with np <= 64 RPL: scaling and Householder product in
// one pass over L_p^{-1}, V and T.  Lane l owns rows l + 64 q (q < RPL) of x_p in
// registers; products whose rows run down a column (L^{-1} x, V u, T w) read the
// matrix with consecutive lanes on consecutive rows, the transposed ones (V^T y,
// T^T w, L^{-T} y) let lane j walk its own column.  The vector being consumed is
// broadcast from LDS.
//   DIR = +1: x_p <- Q_p^T L_p^{-1} x_p      DIR = -1: x_p <- L_p^{-T} Q_p x_p
template <int RPL>
__device__ inline void iface_put(double (*buf)[RB], const double (&v)[RPL][RB]) {
#pragma unroll
  for (int q = 0; q < RPL; ++q)
#pragma unroll
    for (int c = 0; c < RB; ++c) buf[threadIdx.x + 64 * q][c] = v[q][c];
  __syncthreads();
}
__device__ inline void iface_get(const double (*buf)[RB], int k, double (&b)[RB]) {
#pragma unroll
  for (int c = 0; c < RB; ++c) b[c] = buf[k][c];
}

// Products of a matrix M (ld ld, nrows x ncols, restricted to mode 0: every entry,
// 1: the upper triangle row <= column, 2: the lower triangle row >= column) with
// the vector vb broadcast from LDS:
//   COLWALK  out[j] = sum_i M[i + j ld] vb_i   lane j walks column j = lane + 64 q
//   else     out[i] = sum_k M[i + k ld] vb_k   lanes run down column k, row i = lane + 64 q
// The matrix is read in chunks of IFC entries (reads past the end are masked and
// give 0; rows of vb beyond the matrix hold 0); the many waves of a launch hide the
// latency of a chunk.
#define IFC 16
template <int RPL, bool COLWALK>
__device__ inline void iface_chunk(const double* __restrict__ M, int ld, int nrows, int ncols, int mode, int k0,
                                   double (&m)[IFC][RPL]) {
#pragma unroll
  for (int u = 0; u < IFC; ++u)
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int own = threadIdx.x + 64 * q, s = k0 + u;  // own: this lane's column (COLWALK) or row
      const int i = COLWALK ? s : own, j = COLWALK ? own : s;
            const bool on = i < nrows && j < ncols && (mode == 0 || (mode == 1 ? i <= j : i >= j));
      m[u][q] = on ? gld(M + i + (int64_t)j * ld) : 0.0;
    }
}
template <int RPL>
__device__ inline void iface_fma(const double (&m)[IFC][RPL], const double (*vb)[RB], int k0,
                                 double (&out)[RPL][RB]) {
#pragma unroll
  for (int u = 0; u < IFC; ++u) {
    double b[RB];
    iface_get(vb, k0 + u, b);
#pragma unroll
    for (int q = 0; q < RPL; ++q)
#pragma unroll
      for (int c = 0; c < RB; ++c) out[q][c] = fma(m[u][q], b[c], out[q][c]);
  }
}
template <int RPL, bool COLWALK>
__device__ inline void iface_product(const double* __restrict__ M, int ld, int nrows, int ncols, int mode,
                                     const double (*vb)[RB], double (&out)[RPL][RB]) {
#pragma unroll
  for (int q = 0; q < RPL; ++q)
#pragma unroll
    for (int c = 0; c < RB; ++c) out[q][c] = 0.0;
  const int n = COLWALK ? nrows : ncols;  // length of the sum
  for (int k0 = 0; k0 < n; k0 += IFC) {
    double m[IFC][RPL];
    iface_chunk<RPL, COLWALK>(M, ld, nrows, ncols, mode, k0, m);
    iface_fma<RPL>(m, vb, k0, out);
  }
}

template <int DIR, int RPL>
__global__ void __launch_bounds__(64) k_iface(const IfaceAp* __restrict__ ds, ApplyArgs a) {
  __shared__ double xb[64 * RPL][RB];  // vector broadcast: x, then y
  __shared__ double wb[64 * RPL][RB];  // w, then u
  const IfaceAp e = ds[blockIdx.x];
  const int np = e.np, r = e.r;
  const int32_t* sl = a.slot + e.slot_p;
#pragma unroll 1
  for (int c0 = 0; c0 < a.nrhs; c0 += RB) {
    const int nr = min(RB, a.nrhs - c0);
    double x[RPL][RB], y[RPL][RB];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int i = threadIdx.x + 64 * q;
      const int64_t v = i < np ? (int64_t)sl[i] : 0;
#pragma unroll
      for (int c = 0; c < RB; ++c) x[q][c] = (i < np && c < nr) ? a.x[v + (int64_t)(c0 + c) * a.ldx] : 0.0;
    }
    if (DIR > 0) {
      iface_put<RPL>(xb, x);
      iface_product<RPL, false>(e.Linv, e.ldl, np, np, 2, xb, y);  // y = L^{-1} x (lower: i >= k)
    } else {
#pragma unroll
      for (int q = 0; q < RPL; ++q)
#pragma unroll
        for (int c = 0; c < RB; ++c) y[q][c] = x[q][c];
    }
    if (r > 0) {  // y <- Q^T y (DIR +1) or Q y (DIR -1), Q = I - V T V^T
      double w[RPL][RB], u[RPL][RB];
      __syncthreads();
      iface_put<RPL>(xb, y);
      iface_product<RPL, true>(e.V, e.ldv, np, r, 0, xb, w);  // w = V^T y
      iface_put<RPL>(wb, w);
      if (DIR > 0)
        iface_product<RPL, true>(e.T, e.ldt, r, r, 1, wb, u);  // u = T^T w (upper: k <= j)
      else
        iface_product<RPL, false>(e.T, e.ldt, r, r, 1, wb, u);  // u = T w (upper: i <= k)
      __syncthreads();
      iface_put<RPL>(wb, u);
      double vu[RPL][RB];
      iface_product<RPL, false>(e.V, e.ldv, np, r, 0, wb, vu);  // V u
#pragma unroll
      for (int q = 0; q < RPL; ++q)
#pragma unroll
        for (int c = 0; c < RB; ++c) y[q][c] -= vu[q][c];
    }
    if (DIR < 0) {
      __syncthreads();
      iface_put<RPL>(xb, y);
      iface_product<RPL, true>(e.Linv, e.ldl, np, np, 2, xb, y);  // y = L^{-T} y (column j of L^{-1}, rows i >= j)
    }
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int i = threadIdx.x + 64 * q;
      if (i < np) {
        const int64_t v = sl[i];
#pragma unroll
        for (int c = 0; c < RB; ++c)
          if (c < nr) a.x[v + (int64_t)(c0 + c) * a.ldx] = y[q][c];
      }
    }
    __syncthreads();  // xb, wb are rewritten by the next right-hand-side block
  }
}

__global__ void k_gather(const int32_t* __restrict__ nslot, int64_t len, ApplyArgs a) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= len) return;
  const int32_t s = nslot[q];
  for (int c0 = 0; c0 < a.nrhs; c0 += RB) {
    double b[RB];
#pragma unroll
    for (int c = 0; c < RB; ++c) b[c] = c0 + c < a.nrhs ? a.x[s + (int64_t)(c0 + c) * a.ldx] : 0.0;
#pragma unroll
    for (int c = 0; c < RB; ++c)
      if (c0 + c < a.nrhs) a.gbuf[q + (int64_t)(c0 + c) * a.ldg] = b[c];
  }
}

// t = x_s - G_{N_s s}^T x_{N_s} for the 64 columns [k0, k0 + 64) of s: one
// workgroup per column tile and chunk of ELIM_RC rows of G.  With one chunk t goes
// straight into the apply scratch of s; with several, each chunk stores its partial
// sum after t and k_elim_bwd forms t from them in chunk order.
__global__ void __launch_bounds__(AW) k_elim_bwd_gemv(const ElimAp* __restrict__ ds, const ElimTile* __restrict__ tl,
                                                      ApplyArgs a) {
  __shared__ TileShared sh;
  const ElimTile et = tl[blockIdx.x];
  const ElimAp e = ds[et.s];
  const int ns = e.ns, k0 = et.k0;
  const int i0 = et.c * ELIM_RC, i1 = min(e.nN, i0 + ELIM_RC);
  const int32_t* sl = a.slot + e.slot_s;
  const int cc = threadIdx.x & 63, g = threadIdx.x >> 6;
  for (int c0 = 0; c0 < a.nrhs; c0 += RB) {
    const int nr = min(RB, a.nrhs - c0);
    double acc[2] = {0.0, 0.0};
    tile_gemv_t(e.G + i0, e.ld, k0, ns, i1 - i0, a.gbuf + e.slot_N + i0 + (int64_t)c0 * a.ldg, a.ldg, nr, sh, acc);
    const int k = k0 + cc;
    if (k < ns) {
      if (e.nchunk == 1) {
        const int64_t xo = sl[k];
        const double x0 = g < nr ? a.x[xo + (int64_t)(c0 + g) * a.ldx] : 0.0;
        const double x1 = g + 4 < nr ? a.x[xo + (int64_t)(c0 + g + 4) * a.ldx] : 0.0;
        if (g < nr) a.tmp[e.tmp + k + (int64_t)(c0 + g) * a.ldt] = x0 - acc[0];
        if (g + 4 < nr) a.tmp[e.tmp + k + (int64_t)(c0 + g + 4) * a.ldt] = x1 - acc[1];
      } else {
        const int64_t pofs = e.tmp + (int64_t)ns * (1 + et.c) + k;
        if (g < nr) a.tmp[pofs + (int64_t)(c0 + g) * a.ldt] = acc[0];
        if (g + 4 < nr) a.tmp[pofs + (int64_t)(c0 + g + 4) * a.ldt] = acc[1];
      }
    }
  }
}

// x_s = L_s^{-T} t
__global__ void __launch_bounds__(AW) k_elim_bwd(const ElimAp* __restrict__ ds, ApplyArgs a) {
  __shared__ TileShared sh;
  const ElimAp e = ds[blockIdx.x];
  const int32_t* sl = a.slot + e.slot_s;
  if (e.nchunk > 1) {  // t = x_s - sum of the chunk partial sums, in chunk order
    for (int k = threadIdx.x; k < e.ns; k += AW) {
      const int64_t xo = sl[k];
      for (int c0 = 0; c0 < a.nrhs; c0 += RB) {
        double v[RB];
#pragma unroll
        for (int c = 0; c < RB; ++c) v[c] = c0 + c < a.nrhs ? a.x[xo + (int64_t)(c0 + c) * a.ldx] : 0.0;
        for (int q = 0; q < e.nchunk; ++q) {
          const double* pq = a.tmp + e.tmp + (int64_t)e.ns * (1 + q) + k;
#pragma unroll
          for (int c = 0; c < RB; ++c)
            if (c0 + c < a.nrhs) v[c] -= pq[(int64_t)(c0 + c) * a.ldt];
        }
#pragma unroll
        for (int c = 0; c < RB; ++c)
          if (c0 + c < a.nrhs) a.tmp[e.tmp + k + (int64_t)(c0 + c) * a.ldt] = v[c];
      }
    }
    __threadfence_block();
    __syncthreads();
  }
  for (int c0 = 0; c0 < a.nrhs; c0 += RB)
    trsv_bwd(e.L, e.ld, e.Dinv, e.ns, a.tmp + e.tmp + (int64_t)c0 * a.ldt, a.ldt, min(RB, a.nrhs - c0), sh);
  scatter_seg(sl, e.ns, a, e.tmp);
}

void apply_step_forward(const StepDev& s, const ApplyArgs& a, hipStream_t st) {
  if (s.n_elim) hipLaunchKernelGGL(k_elim_fwd, dim3(s.n_elim), dim3(AW), 0, st, s.elim, a);
  if (s.n_ftile) hipLaunchKernelGGL(k_fwd_gemv, dim3(s.n_ftile), dim3(AW), 0, st, s.elim, s.ftile, a);
  if (s.n_target) hipLaunchKernelGGL(k_target_sum, dim3(s.n_target), dim3(AW), 0, st, s.target, s.contrib, a);
  if (s.n_iface1) hipLaunchKernelGGL((k_iface<1, 1>), dim3(s.n_iface1), dim3(64), 0, st, s.iface, a);
  if (s.n_iface2) hipLaunchKernelGGL((k_iface<1, 2>), dim3(s.n_iface2), dim3(64), 0, st, s.iface + s.n_iface1, a);
  if (s.n_stile) {
    hipLaunchKernelGGL(k_gather_rows, dim3((s.sgather_len + 255) / 256), dim3(256), 0, st, s.sgather,
                       s.sgather_len, a);
    hipLaunchKernelGGL(k_scale<1>, dim3(s.n_stile), dim3(AW), 0, st, s.scale, s.stile, a);
  }
  if (s.n_hr) {
    hipLaunchKernelGGL(k_house_w, dim3(s.n_hr), dim3(AW), 0, st, s.house, s.hr, a);
    hipLaunchKernelGGL(k_house_t<1>, dim3(s.n_hr), dim3(AW), 0, st, s.house, s.hr, a);
    hipLaunchKernelGGL(k_house_v, dim3(s.n_hv), dim3(AW), 0, st, s.house, s.hv, a);
  }
  if (s.n_interp) launch_interp_apply(s.interp, s.n_interp, a, 1, st);
}

void apply_step_backward(const StepDev& s, const ApplyArgs& a, hipStream_t st) {
  if (s.n_interp) launch_interp_apply(s.interp, s.n_interp, a, -1, st);
  if (s.n_iface1) hipLaunchKernelGGL((k_iface<-1, 1>), dim3(s.n_iface1), dim3(64), 0, st, s.iface, a);
  if (s.n_iface2) hipLaunchKernelGGL((k_iface<-1, 2>), dim3(s.n_iface2), dim3(64), 0, st, s.iface + s.n_iface1, a);
  if (s.n_hr) {
    hipLaunchKernelGGL(k_house_w, dim3(s.n_hr), dim3(AW), 0, st, s.house, s.hr, a);
    hipLaunchKernelGGL(k_house_t<-1>, dim3(s.n_hr), dim3(AW), 0, st, s.house, s.hr, a);
    hipLaunchKernelGGL(k_house_v, dim3(s.n_hv), dim3(AW), 0, st, s.house, s.hv, a);
  }
  if (s.n_stile) {
    hipLaunchKernelGGL(k_gather_rows, dim3((s.sgather_len + 255) / 256), dim3(256), 0, st, s.sgather,
                       s.sgather_len, a);
    hipLaunchKernelGGL(k_scale<-1>, dim3(s.n_stile), dim3(AW), 0, st, s.scale, s.stile, a);
  }
  if (s.n_elim) {
    if (s.nslot_len)
      hipLaunchKernelGGL(k_gather, dim3((s.nslot_len + 255) / 256), dim3(256), 0, st, s.nslot, s.nslot_len, a);
    if (s.n_etile) hipLaunchKernelGGL(k_elim_bwd_gemv, dim3(s.n_etile), dim3(AW), 0, st, s.elim, s.etile, a);
    hipLaunchKernelGGL(k_elim_bwd, dim3(s.n_elim), dim3(AW), 0, st, s.elim, a);
  }
}

// ---------------------------------------------------------------- PCG vector kernels
// y = A x for up to RB right-hand sides at a time: one row per thread, its entries
// read once per block of right-hand sides.
__global__ void __launch_bounds__(256) k_spmv(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                                              const double* __restrict__ val, int64_t n, int nrhs,
                                              const double* __restrict__ x, double* __restrict__ y, int64_t ld) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t b = rowptr[v], e = rowptr[v + 1];
  for (int c0 = 0; c0 < nrhs; c0 += RB) {
    const int nr = min(RB, nrhs - c0);
    const double* xc = x + (int64_t)c0 * ld;
    double s[RB];
#pragma unroll
    for (int c = 0; c < RB; ++c) s[c] = 0.0;
    // eight entries of the row at a time: their values and columns, then every x
    // entry they need, are requested together (the sum keeps the entries' order)
    for (int64_t q0 = b; q0 < e; q0 += 8) {
      double a[8];
      int64_t col[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool ok = q0 + u < e;
        a[u] = ok ? val[q0 + u] : 0.0;
        col[u] = ok ? (int64_t)colind[q0 + u] : v;
      }
      double xv[8][RB];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int c = 0; c < RB; ++c) xv[u][c] = c < nr ? xc[col[u] + (int64_t)c * ld] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (q0 + u < e) {
#pragma unroll
          for (int c = 0; c < RB; ++c)
            if (c < nr) s[c] = fma(a[u], xv[u][c], s[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < RB; ++c)
      if (c < nr) y[v + (int64_t)(c0 + c) * ld] = s[c];
  }
}

// partial[blk + c*nblk] = sum over this block's rows of a[:,c] * b[:,c]
__global__ void __launch_bounds__(256) k_dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                     int64_t n, double* __restrict__ partial) {
  const int c = blockIdx.y;
  const int64_t nblk = gridDim.x;
  const double* ac = a + (int64_t)c * n;
  const double* bc = b + (int64_t)c * n;
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += nblk * 256) s += ac[i] * bc[i];
  __shared__ double red[4];
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x + (int64_t)c * nblk] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256) k_dot_final(const double* __restrict__ partial, int nblk,
                                                   double* __restrict__ out) {
  const int c = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) s += partial[i + (int64_t)c * nblk];
  __shared__ double red[4];
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[c] = red[0] + red[1] + red[2] + red[3];
}

// alpha_c = active ? rz/pq : 0; x += alpha p; r -= alpha q
__global__ void k_update_xr(int64_t n, int nrhs, const double* __restrict__ rz, const double* __restrict__ pq,
                            const int32_t* __restrict__ active, const double* __restrict__ p,
                            const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < nrhs; ++c) {
    if (!active[c]) continue;
    const double alpha = rz[c] / pq[c];
    const int64_t o = i + (int64_t)c * n;
    x[o] += alpha * p[o];
    r[o] -= alpha * q[o];
  }
}

// p = z + beta p with beta = rz_new/rz (active columns only)
__global__ void k_update_p(int64_t n, int nrhs, const double* __restrict__ rz_new, const double* __restrict__ rz,
                           const int32_t* __restrict__ active, const double* __restrict__ z, double* __restrict__ p) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < nrhs; ++c) {
    if (!active[c]) continue;
    const double beta = rz_new[c] / rz[c];
    const int64_t o = i + (int64_t)c * n;
    p[o] = z[o] + beta * p[o];
  }
}

// z = r (plain copy; a kernel so that the apply can be captured into a graph)
__global__ void k_permute(const double* __restrict__ src, double* __restrict__ dst, const int32_t* __restrict__ idx,
                          int64_t n, int nrhs, int64_t ld) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t from = idx[i];
  for (int c = 0; c < nrhs; ++c) dst[i + (int64_t)c * ld] = src[from + (int64_t)c * ld];
}

void launch_permute(const double* src, double* dst, const int32_t* idx, int64_t n, int nrhs, int64_t ld,
                    hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_permute, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, src, dst, idx, n, nrhs, ld);
}

__global__ void k_copy_vec(const double* __restrict__ r, double* __restrict__ z, int64_t len) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < len) z[i] = r[i];
}

// y = b - y (true residual)
__global__ void k_residual(int64_t len, const double* __restrict__ b, double* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < len) y[i] = b[i] - y[i];
}

void launch_spmv(const int64_t* rowptr, const int32_t* colind, const double* val, int64_t n, int nrhs,
                 const double* x, double* y, hipStream_t s, int64_t ld) {
  hipLaunchKernelGGL(k_spmv, dim3((n + 255) / 256), dim3(256), 0, s, rowptr, colind, val, n, nrhs, x, y,
                     ld > 0 ? ld : n);
}

// ---------------------------------------------------------------- batched PCG kernels
// Several problems stacked in one vector of leading dimension ld (problem q in rows
// [off[q], off[q] + n_q)); scalars per (problem, column) at q * nrhs + c.  The dot
// products keep the single-problem reduction order: problem q has nblk[q] blocks
// (its own count), each summing its rows with the same stride and tree.
__global__ void __launch_bounds__(256) k_seg_dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                         int64_t ld, const SegBlk* __restrict__ blks, int64_t nb_tot,
                                                         double* __restrict__ partial) {
  const int c = blockIdx.y;
  const SegBlk sb = blks[blockIdx.x];
  const double* ac = a + sb.off + (int64_t)c * ld;
  const double* bc = b + sb.off + (int64_t)c * ld;
  double s = 0.0;
  for (int64_t i = int64_t(sb.local) * 256 + threadIdx.x; i < sb.n; i += int64_t(sb.nblk) * 256) s += ac[i] * bc[i];
  __shared__ double red[4];
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x + (int64_t)c * nb_tot] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256) k_seg_dot_final(const double* __restrict__ partial, const int64_t* __restrict__ pbase,
                                                       const int32_t* __restrict__ nblk, int64_t nb_tot, int nrhs,
                                                       double* __restrict__ out) {
  const int q = blockIdx.x, c = blockIdx.y;
  const double* pp = partial + pbase[q] + (int64_t)c * nb_tot;
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk[q]; i += 256) s += pp[i];
  __shared__ double red[4];
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[(int64_t)q * nrhs + c] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_seg_update_xr(int64_t ntot, int nrhs, const int32_t* __restrict__ pid, const double* __restrict__ rz,
                                const double* __restrict__ pq, const int32_t* __restrict__ active,
                                const double* __restrict__ p, const double* __restrict__ q, double* __restrict__ x,
                                double* __restrict__ r) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  const int64_t k = (int64_t)pid[i] * nrhs;
  for (int c = 0; c < nrhs; ++c) {
    if (!active[k + c]) continue;
    const double alpha = rz[k + c] / pq[k + c];
    const int64_t o = i + (int64_t)c * ntot;
    x[o] += alpha * p[o];
    r[o] -= alpha * q[o];
  }
}

__global__ void k_seg_update_p(int64_t ntot, int nrhs, const int32_t* __restrict__ pid, const double* __restrict__ rz_new,
                               const double* __restrict__ rz, const int32_t* __restrict__ active,
                               const double* __restrict__ z, double* __restrict__ p) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  const int64_t k = (int64_t)pid[i] * nrhs;
  for (int c = 0; c < nrhs; ++c) {
    if (!active[k + c]) continue;
    const double beta = rz_new[k + c] / rz[k + c];
    const int64_t o = i + (int64_t)c * ntot;
    p[o] = z[o] + beta * p[o];
  }
}

// y = A x for every problem of a stacked vector (leading dimension ld): one thread per
// row, 256-row blocks of one problem each; the same per-row arithmetic as k_spmv.
__global__ void __launch_bounds__(256) k_spmv_batch(const SpmvProb* __restrict__ probs, const int2* __restrict__ blk,
                                                    int nrhs, int64_t ld, const double* __restrict__ x,
                                                    double* __restrict__ y) {
  const int2 bq = blk[blockIdx.x];
  const SpmvProb pr = probs[bq.x];
  const int64_t v = int64_t(bq.y) * 256 + threadIdx.x;
  if (v >= pr.n) return;
  const int64_t b = pr.rowptr[v], e = pr.rowptr[v + 1];
  const double* xo = x + pr.off;
  for (int c0 = 0; c0 < nrhs; c0 += RB) {
    const int nr = min(RB, nrhs - c0);
    const double* xc = xo + (int64_t)c0 * ld;
    double s[RB];
#pragma unroll
    for (int c = 0; c < RB; ++c) s[c] = 0.0;
    for (int64_t q = b; q < e; ++q) {
      const double a = pr.val[q];
      const int64_t col = pr.colind[q];
#pragma unroll
      for (int c = 0; c < RB; ++c)
        if (c < nr) s[c] = fma(a, xc[col + (int64_t)c * ld], s[c]);
    }
#pragma unroll
    for (int c = 0; c < RB; ++c)
      if (c < nr) y[pr.off + v + (int64_t)(c0 + c) * ld] = s[c];
  }
}

// Copies between each problem's own n x nrhs block (leading dimension n) and its rows
// of the stacked vector (leading dimension ld); TO_STACK selects the direction.
template <bool TO_STACK>
__global__ void k_stack(const StackProb* __restrict__ probs, const int2* __restrict__ blk, int nrhs, int64_t ld,
                        double* __restrict__ stacked) {
  const int2 bq = blk[blockIdx.x];
  const StackProb pr = probs[bq.x];
  const int64_t v = int64_t(bq.y) * 256 + threadIdx.x;
  if (v >= pr.n) return;
  for (int c = 0; c < nrhs; ++c) {
    if (TO_STACK)
      stacked[pr.off + v + (int64_t)c * ld] = pr.own_in[v + (int64_t)c * pr.n];
    else
      pr.own_out[v + (int64_t)c * pr.n] = stacked[pr.off + v + (int64_t)c * ld];
  }
}

void launch_spmv_batch(const SpmvProb* probs, const int2* blk, int64_t nblk, int nrhs, int64_t ld, const double* x,
                       double* y, hipStream_t s) {
  if (nblk > 0) hipLaunchKernelGGL(k_spmv_batch, dim3(nblk), dim3(256), 0, s, probs, blk, nrhs, ld, x, y);
}
void launch_stack(const StackProb* probs, const int2* blk, int64_t nblk, int nrhs, int64_t ld, double* stacked,
                  bool to_stack, hipStream_t s) {
  if (nblk == 0) return;
  if (to_stack)
    hipLaunchKernelGGL(k_stack<true>, dim3(nblk), dim3(256), 0, s, probs, blk, nrhs, ld, stacked);
  else
    hipLaunchKernelGGL(k_stack<false>, dim3(nblk), dim3(256), 0, s, probs, blk, nrhs, ld, stacked);
}

void launch_seg_dot(const double* a, const double* b, int64_t ld, int nrhs, const SegBlk* blks, int64_t nb_tot,
                    const int64_t* pbase, const int32_t* nblk, int32_t P, double* partial, double* out,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_seg_dot_partial, dim3(nb_tot, nrhs), dim3(256), 0, s, a, b, ld, blks, nb_tot, partial);
  hipLaunchKernelGGL(k_seg_dot_final, dim3(P, nrhs), dim3(256), 0, s, partial, pbase, nblk, nb_tot, nrhs, out);
}
void launch_seg_update_xr(int64_t ntot, int nrhs, const int32_t* pid, const double* rz, const double* pq,
                          const int32_t* active, const double* p, const double* q, double* x, double* r, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_update_xr, dim3((ntot + 255) / 256), dim3(256), 0, s, ntot, nrhs, pid, rz, pq, active, p, q,
                     x, r);
}
void launch_seg_update_p(int64_t ntot, int nrhs, const int32_t* pid, const double* rz_new, const double* rz,
                         const int32_t* active, const double* z, double* p, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_update_p, dim3((ntot + 255) / 256), dim3(256), 0, s, ntot, nrhs, pid, rz_new, rz, active,
                     z, p);
}
void launch_dot(const double* a, const double* b, int64_t n, int nrhs, double* partial, int nblk, double* out,
                hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(nblk, nrhs), dim3(256), 0, s, a, b, n, partial);
  hipLaunchKernelGGL(k_dot_final, dim3(nrhs), dim3(256), 0, s, partial, nblk, out);
}
void launch_update_xr(int64_t n, int nrhs, const double* rz, const double* pq, const int32_t* active,
                      const double* p, const double* q, double* x, double* r, hipStream_t s) {
  hipLaunchKernelGGL(k_update_xr, dim3((n + 255) / 256), dim3(256), 0, s, n, nrhs, rz, pq, active, p, q, x, r);
}
void launch_update_p(int64_t n, int nrhs, const double* rz_new, const double* rz, const int32_t* active,
                     const double* z, double* p, hipStream_t s) {
  hipLaunchKernelGGL(k_update_p, dim3((n + 255) / 256), dim3(256), 0, s, n, nrhs, rz_new, rz, active, z, p);
}
void launch_copy_vec(const double* r, double* z, int64_t len, hipStream_t s) {
  if (len > 0) hipLaunchKernelGGL(k_copy_vec, dim3((len + 255) / 256), dim3(256), 0, s, r, z, len);
}
void launch_residual(int64_t len, const double* b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3((len + 255) / 256), dim3(256), 0, s, len, b, y);
}

}  // namespace spand
