// 64x64 complex GEMM tile on the gfx950 matrix cores (planar complex, column-major).
//
// A work-group of 256 threads (4 wave64s) computes C[64x64] += A[64xK] * B[Kx64] with
// K a multiple of 16.  Operands are staged through LDS in 16-deep slabs (double
// buffered: the next slab is fetched into registers while the current one feeds the
// MFMAs).  Each wave owns a 32x32 quadrant as 2x2 tiles of v_mfma_*_16x16x4; a complex
// product is four real MFMAs: Re += Ar*Br - Ai*Bi, Im += Ar*Bi + Ai*Br.
// MFMA 16x16x4 operand layout: lane l supplies A[l%16][l/16] and B[l/16][l%16].  The
// accumulator element v of lane l is D[4*(l/16)+v][l%16] for the FP32 instruction and
// D[(l/16)+4v][l%16] for the FP64 one (measured on gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace qoc {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T> struct Vec4;
template <> struct Vec4<double> { typedef d4v type; };
template <> struct Vec4<float> { typedef f4v type; };

__device__ inline d4v mfma16(double a, double b, d4v c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline f4v mfma16(float a, float b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

constexpr int TBM = 64, TBN = 64, TBK = 16;
constexpr int TPAD = 4;  // LDS row padding (elements)

template <typename T>
struct TileLds {
  T a[2][2][TBK][TBM + TPAD];  // [buffer][plane][k][row]
  T b[2][2][TBK][TBN + TPAD];  // [buffer][plane][k][col]
};

template <typename T>
struct TileAcc {
  typename Vec4<T>::type re[2][2];
  typename Vec4<T>::type im[2][2];
};

// Operand pointers of one tile product.  Planes: re at p, im at p + plane stride.
template <typename T>
struct TileOperands {
  const T* A;
  long long a_ps;
  int lda;
  const T* B;
  long long b_ps;
  int ldb;
  int M, N, K;   // M, N, K multiples of 16
  int row0, col0;
};

template <typename T>
__device__ inline void tile_fetch(const TileOperands<T>& op, int k0, T (&ra)[8], T (&rb)[8]) {
  const int t = threadIdx.x;
  const int plane = t >> 7, tt = t & 127;
  {  // A: 8 consecutive rows of one k column
    const int kk = tt >> 3, ii = (tt & 7) * 8;
    const int row = op.row0 + ii;
    if (row < op.M) {
      const T* p = op.A + plane * op.a_ps + (long long)(k0 + kk) * op.lda + row;
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[e] = p[e];
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[e] = T(0);
    }
  }
  {  // B: 8 consecutive k of one column
    const int jj = tt >> 1, kk = (tt & 1) * 8;
    const int col = op.col0 + jj;
    if (col < op.N) {
      const T* p = op.B + plane * op.b_ps + (long long)col * op.ldb + k0 + kk;
#pragma unroll
      for (int e = 0; e < 8; ++e) rb[e] = p[e];
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) rb[e] = T(0);
    }
  }
}

template <typename T>
__device__ inline void tile_stash(TileLds<T>& s, int buf, const T (&ra)[8], const T (&rb)[8]) {
  const int t = threadIdx.x;
  const int plane = t >> 7, tt = t & 127;
  {
    const int kk = tt >> 3, ii = (tt & 7) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) s.a[buf][plane][kk][ii + e] = ra[e];
  }
  {
    const int jj = tt >> 1, kk = (tt & 1) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) s.b[buf][plane][kk + e][jj] = rb[e];
  }
}

// Full K loop for one 64x64 output tile; acc is zeroed here.
template <typename T>
__device__ inline void tile_mma(const TileOperands<T>& op, TileLds<T>& s, TileAcc<T>& acc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  bool rv[2], cv[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    rv[q] = op.row0 + wr * 32 + q * 16 < op.M;
    cv[q] = op.col0 + wc * 32 + q * 16 < op.N;
  }
#pragma unroll
  for (int ri = 0; ri < 2; ++ri)
#pragma unroll
    for (int ci = 0; ci < 2; ++ci) {
      acc.re[ri][ci] = typename Vec4<T>::type{0, 0, 0, 0};
      acc.im[ri][ci] = typename Vec4<T>::type{0, 0, 0, 0};
    }
  T ra[8], rb[8];
  const int nk = op.K / TBK;
  tile_fetch(op, 0, ra, rb);
  __syncthreads();  // previous users of the LDS buffers are done
  tile_stash(s, 0, ra, rb);
  __syncthreads();
  for (int kb = 0; kb < nk; ++kb) {
    const int buf = kb & 1;
    if (kb + 1 < nk) tile_fetch(op, (kb + 1) * TBK, ra, rb);
#pragma unroll
    for (int k4 = 0; k4 < TBK / 4; ++k4) {
      const int kq = k4 * 4 + (lane >> 4);
      const int rr = lane & 15;
      T ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        ar[q] = s.a[buf][0][kq][wr * 32 + q * 16 + rr];
        ai[q] = s.a[buf][1][kq][wr * 32 + q * 16 + rr];
        br[q] = s.b[buf][0][kq][wc * 32 + q * 16 + rr];
        bi[q] = s.b[buf][1][kq][wc * 32 + q * 16 + rr];
      }
#pragma unroll
      for (int ri = 0; ri < 2; ++ri) {
        if (!rv[ri]) continue;
#pragma unroll
        for (int ci = 0; ci < 2; ++ci) {
          if (!cv[ci]) continue;
          acc.re[ri][ci] = mfma16(ar[ri], br[ci], acc.re[ri][ci]);
          acc.re[ri][ci] = mfma16(-ai[ri], bi[ci], acc.re[ri][ci]);
          acc.im[ri][ci] = mfma16(ar[ri], bi[ci], acc.im[ri][ci]);
          acc.im[ri][ci] = mfma16(ai[ri], br[ci], acc.im[ri][ci]);
        }
      }
    }
    if (kb + 1 < nk) {
      tile_stash(s, buf ^ 1, ra, rb);
    }
    __syncthreads();
  }
}

// First row of sub-tile ri of this wave, and the row offset of accumulator element v.
__device__ inline int acc_row_base(int row0, int ri) {
  const int wave = threadIdx.x >> 6;
  return row0 + (wave >> 1) * 32 + ri * 16;
}
template <typename T> __device__ inline int acc_row_off(int v);
template <> __device__ inline int acc_row_off<float>(int v) { return 4 * ((threadIdx.x & 63) >> 4) + v; }
template <> __device__ inline int acc_row_off<double>(int v) { return ((threadIdx.x & 63) >> 4) + 4 * v; }
__device__ inline int acc_col(int col0, int ci) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return col0 + (wave & 1) * 32 + ci * 16 + (lane & 15);
}

// Persistent scheduling: work-group w runs on XCD w % 8; each XCD takes a contiguous
// eighth of the item space so that tiles of one matrix share that XCD's L2.
struct ItemRange {
  long long begin, end, step;
};
__device__ inline ItemRange xcd_items(long long total) {
  const int G = gridDim.x;
  const int w = blockIdx.x;
  const int nx = G >= 8 ? 8 : 1;
  const int x = w % nx;
  const int per_x = G / nx;
  const int lw = w / nx;
  const long long chunk = (total + nx - 1) / nx;
  ItemRange r;
  r.begin = (long long)x * chunk + lw;
  r.end = (long long)(x + 1) * chunk;
  if (r.end > total) r.end = total;
  r.step = per_x;
  if (lw >= per_x) r.begin = r.end;  // grid not a multiple of 8: spare groups idle
  return r;
}

}  // namespace qoc
