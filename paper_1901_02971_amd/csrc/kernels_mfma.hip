// Batched variable-size GEMM on the CDNA4 matrix cores.
//
// Descriptors built by the host, expanded on the device into a tile -> product map:
// one 64x64 output tile per workgroup of 4
// waves; wave (wm, wn) owns the 32x32 quadrant (wm, wn) as 2x2 blocks of 16x16
// MFMA outputs.  Operand tiles are staged k-major in LDS so that the 16 lanes
// reading one fragment touch consecutive addresses.
//
//   MODE 0  FP64 operands, v_mfma_f64_16x16x4f64, FP64 accumulation
//   MODE 1  operands rounded to FP32, v_mfma_f32_16x16x4f32, FP32 accumulation
//   MODE 2  BF16x3: each FP32-rounded operand is split a = hi + lo (hi = bf16(a),
//           lo = bf16(a - hi)); a*b ~ hi*hi + hi*lo + lo*hi with
//           v_mfma_f32_16x16x32_bf16, FP32 accumulation (the split product of
//           Henry, Tang and Heinecke, ARITH 2019)
//
// Lane layout of the 16x16 blocks (lane l, 0..63): A fragment row l%16, k-group
// l/16; B fragment column l%16, k-group l/16; accumulator layout in store_blocks.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.h"

namespace spand {

#define MW 256

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

namespace {

// Operand entries outside the product read a zero constant instead of branching
// around the load, so that a thread's loads are all in flight together.
__device__ const double g_gemm_zero[1] = {0.0};
typedef __attribute__((address_space(1))) const double gdouble_m;
typedef __attribute__((address_space(1))) double gdouble_mw;
__device__ inline double gldm(const double* p) { return *(gdouble_m*)p; }

__device__ inline double load_a(const GemmDesc& d, int gm, int gk, int kmax) {
  const bool ok = !(gm >= d.M || gk >= kmax || ((d.flags & G_TRIA) && gk > gm));
  const double* p = (d.flags & G_TA) ? d.A + gk + (int64_t)gm * d.lda : d.A + gm + (int64_t)gk * d.lda;
  return gldm(ok ? p : g_gemm_zero);
}
__device__ inline double load_b(const GemmDesc& d, int gk, int gn, int kmax) {
  const bool ok = !(gn >= d.N || gk >= kmax || ((d.flags & G_TRIB) && gk > gn));
  const double* p = (d.flags & G_TB) ? d.B + gn + (int64_t)gk * d.ldb : d.B + gk + (int64_t)gn * d.ldb;
  return gldm(ok ? p : g_gemm_zero);
}

// Global -> LDS index of element q (0..TS*BK) of a TS x BK operand tile, chosen so
// that consecutive threads read consecutive global addresses.
template <int TS = 64>
__device__ inline void tile_index(bool trans_major, int q, int BK, int& mm, int& kk) {
  if (!trans_major) { mm = q % TS; kk = q / TS; } else { kk = q % BK; mm = q / BK; }
}

// Accumulator entry i of lane l sits at column l%16 and row 4*(l/16)+i for the
// FP32-accumulating instructions but at row l/16+4*i for v_mfma_f64_16x16x4f64
// (both measured on gfx950).
// C <- alpha acc + beta C over the four 16 x 16 blocks of a wave: every read of C
// (from a clamped address) is issued before the first store.
template <bool F64, typename C4, int PM = 2, int PN = 2>
__device__ inline void store_blocks(const GemmDesc& d, int row0, int col0, const C4 (&acc)[PM][PN]) {
  const int lane = threadIdx.x & 63;
  // two block rows at a time (all of them for the 64 x 64 tile): every read of C of
  // the pair is issued before its first store, without holding the whole tile live
#pragma unroll
  for (int p0 = 0; p0 < PM; p0 += 2) {
    constexpr int PR = PM < 2 ? PM : 2;
    double cv[PR][PN][4];
    int64_t off[PR][PN][4];
    bool ok[PR][PN][4];
#pragma unroll
    for (int pp = 0; pp < PR; ++pp)
#pragma unroll
      for (int q = 0; q < PN; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int p = p0 + pp;
          const int gn = col0 + q * 16 + (lane & 15);
          const int gm = row0 + p * 16 + (F64 ? (lane >> 4) + 4 * i : 4 * (lane >> 4) + i);
          ok[pp][q][i] = gm < d.M && gn < d.N;
          off[pp][q][i] = ok[pp][q][i] ? gm + (int64_t)gn * d.ldc : 0;
        }
    if (d.beta != 0.0) {
#pragma unroll
      for (int pp = 0; pp < PR; ++pp)
#pragma unroll
        for (int q = 0; q < PN; ++q)
#pragma unroll
          for (int i = 0; i < 4; ++i) cv[pp][q][i] = gldm(d.C + off[pp][q][i]);
    }
#pragma unroll
    for (int pp = 0; pp < PR; ++pp)
#pragma unroll
      for (int q = 0; q < PN; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (!ok[pp][q][i]) continue;
          double v = d.alpha * (double)acc[p0 + pp][q][i];
          if (d.beta != 0.0) v += d.beta * cv[pp][q][i];
          *(gdouble_mw*)(d.C + off[pp][q][i]) = v;
        }
  }
}

// Tile (row, column) of the local-th output tile of a product: row-major over all
// tiles, or row-major over the lower triangle (part 1), or its transpose (part 2).
__device__ inline void tile_coords(const GemmDesc& d, int64_t local, int& tm, int& tn, int TS = 64) {
  if (d.part == 0) {
    const int64_t ntn = (d.N + TS - 1) / TS;
    tm = (int)(local / ntn);
    tn = (int)(local - (int64_t)tm * ntn);
    return;
  }
  int a = (int)((sqrt(8.0 * (double)local + 1.0) - 1.0) * 0.5);
  while ((int64_t)(a + 1) * (a + 2) / 2 <= local) ++a;
  while ((int64_t)a * (a + 1) / 2 > local) --a;
  const int b = (int)(local - (int64_t)a * (a + 1) / 2);
  if (d.part == 1) {
    tm = a;
    tn = b;
  } else {
    tm = b;
    tn = a;
  }
}

}  // namespace

// MODE 0 / 1: one TS x TS output tile per workgroup of 4 waves, wave (wm, wn) owning
// the (TS/2) x (TS/2) quadrant as (TS/32) x (TS/32) blocks of 16 x 16 MFMA outputs.
// K is staged BK at a time (the next stage read into registers while the current one
// is multiplied), BK/4 k=4 MFMA steps per stage.  Every tile shape adds the products
// of an output entry in the same k order, so all shapes give the same bits.
template <int MODE, int TS, int BK>
__global__ void __launch_bounds__(MW) k_gemm_mfma(const GemmDesc* __restrict__ descs,
                                                  const int32_t* __restrict__ tile_desc, int64_t tile0) {
  typedef typename std::conditional<MODE == 0, double, float>::type T;
  typedef typename std::conditional<MODE == 0, d4_t, f4_t>::type C4;
  constexpr int PER = TS * BK / MW;  // operand entries per thread and stage
  constexpr int PB = TS / 32;        // 16 x 16 blocks per wave and dimension
  __shared__ T As[BK][TS + 1];
  __shared__ T Bs[BK][TS + 1];
  const int64_t tile = tile0 + blockIdx.x;
  const GemmDesc d = descs[tile_desc[tile]];
  int tmi, tni;
  tile_coords(d, tile - d.t0, tmi, tni, TS);
  const int m0 = tmi * TS, n0 = tni * TS;
  int kmax = d.K;
  if (d.flags & G_TRIA) kmax = min(kmax, m0 + TS);
  if (d.flags & G_TRIB) kmax = min(kmax, n0 + TS);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  C4 acc[PB][PB];
#pragma unroll
  for (int a = 0; a < PB; ++a)
#pragma unroll
    for (int b = 0; b < PB; ++b) acc[a][b] = C4{0, 0, 0, 0};
  const bool ta = d.flags & G_TA, tb = d.flags & G_TB;
  // the next stage is read into registers while the current one is multiplied
  T ra[PER], rb[PER];
  auto load_stage = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = threadIdx.x + u * MW;
      int mm, kk, nn, kb;
      tile_index<TS>(ta, q, BK, mm, kk);
      tile_index<TS>(!tb, q, BK, nn, kb);
      ra[u] = (T)load_a(d, m0 + mm, k0 + kk, kmax);
      rb[u] = (T)load_b(d, k0 + kb, n0 + nn, kmax);
    }
  };
  if (kmax > 0) load_stage(0);
  for (int k0 = 0; k0 < kmax; k0 += BK) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = threadIdx.x + u * MW;
      int mm, kk, nn, kb;
      tile_index<TS>(ta, q, BK, mm, kk);
      tile_index<TS>(!tb, q, BK, nn, kb);
      As[kk][mm] = ra[u];
      Bs[kb][nn] = rb[u];
    }
    __syncthreads();
    if (k0 + BK < kmax) load_stage(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + (lane >> 4);
      T a[PB], b[PB];
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        a[q] = As[kk][wm * (TS / 2) + q * 16 + (lane & 15)];
        b[q] = Bs[kk][wn * (TS / 2) + q * 16 + (lane & 15)];
      }
#pragma unroll
      for (int p = 0; p < PB; ++p)
#pragma unroll
        for (int q = 0; q < PB; ++q) {
          if constexpr (MODE == 0)
            acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], acc[p][q], 0, 0, 0);
          else
            acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[p], b[q], acc[p][q], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  store_blocks<MODE == 0, C4, PB, PB>(d, m0 + wm * (TS / 2), n0 + wn * (TS / 2), acc);
}

// MODE 2 (BF16x3): K staged 32 at a time, one k=32 step (three MFMAs) per stage.
__global__ void __launch_bounds__(MW) k_gemm_bf16x3(const GemmDesc* __restrict__ descs,
                                                    const int32_t* __restrict__ tile_desc, int64_t tile0) {
  constexpr int BK = 32;
  constexpr int LDK = BK + 8;  // row pitch in bf16 (80 bytes)
  __shared__ __attribute__((aligned(16))) __bf16 Ah[64 * LDK], Al[64 * LDK], Bh[64 * LDK], Bl[64 * LDK];
  const int64_t tile = tile0 + blockIdx.x;
  const GemmDesc d = descs[tile_desc[tile]];
  int tmi, tni;
  tile_coords(d, tile - d.t0, tmi, tni);
  const int m0 = tmi * 64, n0 = tni * 64;
  int kmax = d.K;
  if (d.flags & G_TRIA) kmax = min(kmax, m0 + 64);
  if (d.flags & G_TRIB) kmax = min(kmax, n0 + 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  f4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4_t{0, 0, 0, 0};
  const bool ta = d.flags & G_TA, tb = d.flags & G_TB;
  for (int k0 = 0; k0 < kmax; k0 += BK) {
    for (int q = threadIdx.x; q < 64 * BK; q += MW) {
      int mm, kk;
      tile_index(ta, q, BK, mm, kk);
      const float a = (float)load_a(d, m0 + mm, k0 + kk, kmax);
      const __bf16 ah = (__bf16)a;
      Ah[mm * LDK + kk] = ah;
      Al[mm * LDK + kk] = (__bf16)(a - (float)ah);
      int nn, kb;
      tile_index(!tb, q, BK, nn, kb);
      const float b = (float)load_b(d, k0 + kb, n0 + nn, kmax);
      const __bf16 bh = (__bf16)b;
      Bh[nn * LDK + kb] = bh;
      Bl[nn * LDK + kb] = (__bf16)(b - (float)bh);
    }
    __syncthreads();
    const int kof = 8 * (lane >> 4);
    bf8_t ahi[2], alo[2], bhi[2], blo[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int ra = (wm * 32 + q * 16 + (lane & 15)) * LDK + kof;
      const int rb = (wn * 32 + q * 16 + (lane & 15)) * LDK + kof;
      ahi[q] = *reinterpret_cast<const bf8_t*>(Ah + ra);
      alo[q] = *reinterpret_cast<const bf8_t*>(Al + ra);
      bhi[q] = *reinterpret_cast<const bf8_t*>(Bh + rb);
      blo[q] = *reinterpret_cast<const bf8_t*>(Bl + rb);
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[p], bhi[q], acc[p][q], 0, 0, 0);
        acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[p], blo[q], acc[p][q], 0, 0, 0);
        acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[p], bhi[q], acc[p][q], 0, 0, 0);
      }
    __syncthreads();
  }
  store_blocks<false>(d, m0 + wm * 32, n0 + wn * 32, acc);
}

__global__ void k_expand_tiles(const GemmDesc* __restrict__ descs, int32_t* __restrict__ tile_desc) {
  const GemmDesc d = descs[blockIdx.x];
  const int64_t n = gemm_tiles(d.M, d.N, d.part, d.ts);
  for (int64_t q = threadIdx.x; q < n; q += blockDim.x) tile_desc[d.t0 + q] = (int32_t)blockIdx.x;
}

void launch_expand_tiles(const GemmDesc* d, int32_t nd, int32_t* tile_desc, hipStream_t s) {
  if (nd > 0) hipLaunchKernelGGL(k_expand_tiles, dim3(nd), dim3(64), 0, s, d, tile_desc);
}

// Output tile of every variant of the FP64 / FP32 GEMM (the BF16x3 one is 64).
int gemm_variant_count() { return 3; }
int gemm_variant_tile(int v) { return v == 1 ? 128 : (v == 2 ? 32 : 64); }

void launch_gemm(const GemmDesc* d, const int32_t* tile_desc, int64_t tile0, int64_t ntiles, int prec,
                 int variant, hipStream_t s) {
  if (ntiles == 0) return;
  const int ts = prec == 2 ? 64 : gemm_variant_tile(variant);
#define GEMM_L(MODE, TS, BK) hipLaunchKernelGGL((k_gemm_mfma<MODE, TS, BK>), dim3(ntiles), dim3(MW), 0, s, d, tile_desc, tile0)
  if (prec == 2) {
    hipLaunchKernelGGL(k_gemm_bf16x3, dim3(ntiles), dim3(MW), 0, s, d, tile_desc, tile0);
  } else if (prec == 0) {
    if (ts == 128) GEMM_L(0, 128, 16);
    else if (ts == 32) GEMM_L(0, 32, 32);
    else GEMM_L(0, 64, 32);
  } else {
    if (ts == 128) GEMM_L(1, 128, 16);
    else if (ts == 32) GEMM_L(1, 32, 32);
    else GEMM_L(1, 64, 32);
  }
#undef GEMM_L
}

}  // namespace spand
