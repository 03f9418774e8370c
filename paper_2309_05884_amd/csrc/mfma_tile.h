// Complex GEMM tile on the gfx950 matrix cores (planar complex, column-major).
//
// A work-group of 256 threads (4 wave64s in a 2x2 arrangement) computes
// C[BM x BN] = A[BM x K] * B[K x BN], K a multiple of 16.  Each wave owns a
// (BM/2) x (BN/2) quadrant as SM x SN sub-tiles of v_mfma_*_16x16x4, and each complex
// multiply-add is built from real MFMAs.  The tile shape is a template parameter
// (TileShape); the library compiles a few shapes per precision and a plan picks one,
// by default or by timing them on its own work (qoc_plan_autotune).
// The complex product takes three real MFMAs per sub-tile and k step instead of four
// (Gauss's 3M form, see TileAcc).
// Operands are staged through double-buffered LDS in 16-deep slabs; the next slab is
// loaded into registers while the current one feeds the MFMAs, and in a persistent loop
// the next tile's first slab is loaded during the current tile's last one.
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

// Work-group tile shape: 4 waves in a 2 x 2 arrangement, each owning SM x SN 16 x 16
// sub-tiles, so the work-group computes BM x BN = 32 SM x 32 SN.  WAVES is the occupancy
// the kernels are compiled for (waves per SIMD).  LDS rows carry PAD elements of
// padding: consecutive k rows of a slab start 16 (FP32) or 32 (FP64) banks apart.
template <typename T_, int SM_, int SN_, int WAVES_>
struct TileShape {
  typedef T_ T;
  static constexpr int SM = SM_, SN = SN_, BM = 32 * SM_, BN = 32 * SN_, PAD = 16, WAVES = WAVES_;
};
constexpr int TBK = 16;

template <typename C>
struct alignas(16) TileLds {
  typename C::T a[2][2][TBK][C::BM + C::PAD];  // [buffer][plane][k][row]
  typename C::T b[2][2][TBK][C::BN + C::PAD];  // [buffer][plane][k][col]
};

// Accumulators.  Inside the K loop the complex product is formed with three real products
// (Gauss): re = Ar*Br, x = Ai*Bi, im = (Ar+Ai)*(Br+Bi); tile_mma returns
// re = Ar*Br - Ai*Bi and im = (Ar+Ai)*(Br+Bi) - Ar*Br - Ai*Bi.
template <typename C>
struct TileAcc {
  typename Vec4<typename C::T>::type re[C::SM][C::SN];
  typename Vec4<typename C::T>::type im[C::SM][C::SN];
  typename Vec4<typename C::T>::type x[C::SM][C::SN];
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

// 16-byte vectors of the working type (4 floats, 2 doubles): clang vector types, so that
// a copy is a vector load or store (HIP's float4 is a struct, copied with memcpy, which
// keeps an array of them out of registers).
typedef double d2v __attribute__((ext_vector_type(2)));
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef f4v type; static constexpr int n = 4; };
template <> struct Vec16<double> { typedef d2v type; static constexpr int n = 2; };

// Slab loads, 16-byte vectors, thread t handles plane t/128 (tt = t%128):
//  A (BM x 16): vectors f = tt + 128 i (i < NA): k = f / CV, rows (f % CV) * VEC .. with
//    CV = BM/VEC vectors per k row; a wave's stores to LDS cover whole k rows.  CV divides
//    128, so a lane's NA vectors share their rows and sit 128/CV k rows apart;
//  B (16 x BN): column tt%BN, KB = BN/8 consecutive k from (tt/BN)*KB (NB vectors); the
//    lanes of a wave store to consecutive columns of one k row (no LDS bank conflicts).
template <typename C>
struct SlabShape {
  static constexpr int VEC = Vec16<typename C::T>::n;
  static constexpr int CV = C::BM / VEC;
  static constexpr int NA = C::BM * TBK / (128 * VEC);
  static constexpr int KB = C::BN / 8;
  static constexpr int NB = KB / VEC;
  static constexpr int TPC = TBK / KB;
  static_assert(NA >= 1 && NB >= 1 && TBK % KB == 0 && 128 % CV == 0, "slab mapping");
};

template <typename C>
struct SlabRegs {
  typename Vec16<typename C::T>::type a[SlabShape<C>::NA];
  typename Vec16<typename C::T>::type b[SlabShape<C>::NB];
};

// This lane's source addresses for the next slab of one tile product.  Rows of A at or
// beyond M and columns of B at or beyond N (edge tiles) are read from the last valid
// row / column instead: those values reach only outputs that are never stored, and every
// load stays inside the operands, with no branch in the K loop.
template <typename C>
struct SlabSrc {
  const typename C::T* a;  // A vector 0; vector i is 128/CV k rows further
  const typename C::T* b;  // first B vector; the NB vectors are consecutive
};

template <typename C>
__device__ inline SlabSrc<C> slab_src(const TileOperands<typename C::T>& op) {
  typedef SlabShape<C> S;
  const int t = threadIdx.x;
  const int plane = t >> 7, tt = t & 127;
  int row = op.row0 + (tt % S::CV) * S::VEC;
  row = row < op.M ? row : op.M - S::VEC;
  int col = op.col0 + tt % C::BN;
  col = col < op.N ? col : op.N - 1;
  SlabSrc<C> p;
  p.a = op.A + plane * op.a_ps + (long long)(tt / S::CV) * op.lda + row;
  p.b = op.B + plane * op.b_ps + (long long)col * op.ldb + (tt / C::BN) * S::KB;
  return p;
}

// Operands live in global memory; saying so keeps the loads off the flat path (whose
// completion the LDS wait counter would then also track).
template <typename V>
__device__ inline V ld_global(const void* p) {
  return *(const __attribute__((address_space(1))) V*)p;
}

template <typename C>
__device__ inline void slab_fetch(const SlabSrc<C>& p, int lda, SlabRegs<C>& r) {
  typedef typename Vec16<typename C::T>::type V;
  typedef SlabShape<C> S;
  const long long ai = (long long)(128 / S::CV) * lda;
#pragma unroll
  for (int i = 0; i < S::NA; ++i) r.a[i] = ld_global<V>(p.a + i * ai);
#pragma unroll
  for (int i = 0; i < S::NB; ++i) r.b[i] = ld_global<V>(p.b + i * S::VEC);
}

template <typename C>
__device__ inline void slab_advance(SlabSrc<C>& p, int lda) {
  p.a += (long long)TBK * lda;
  p.b += TBK;
}

// Load slab 0 of a tile product into r.
template <typename C>
__device__ inline void tile_prime(const TileOperands<typename C::T>& op, SlabRegs<C>& r) {
  slab_fetch<C>(slab_src<C>(op), op.lda, r);
}

template <typename C>
__device__ inline void tile_stash(TileLds<C>& s, int buf, const SlabRegs<C>& r) {
  typedef typename Vec16<typename C::T>::type V;
  typedef SlabShape<C> S;
  const int t = threadIdx.x;
  const int plane = t >> 7, tt = t & 127;
#pragma unroll
  for (int i = 0; i < S::NA; ++i) {
    const int f = tt + 128 * i;
    *static_cast<V*>(__builtin_assume_aligned(&s.a[buf][plane][f / S::CV][(f % S::CV) * S::VEC], 16)) = r.a[i];
  }
  const int jj = tt % C::BN, kk = (tt / C::BN) * S::KB;
#pragma unroll
  for (int i = 0; i < S::NB; ++i)
#pragma unroll
    for (int e = 0; e < S::VEC; ++e) s.b[buf][plane][kk + i * S::VEC + e][jj] = r.b[i][e];
}

// Wave placement inside the work-group tile (the wave index is uniform: a scalar).
__device__ inline int tile_wave() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// MFMA operands of one 4-deep k step: this lane's rows of A and columns of B.
template <typename C>
struct StepOps {
  typename C::T ar[C::SM], ai[C::SM], br[C::SN], bi[C::SN];
};

template <typename C>
__device__ inline void step_load(const TileLds<C>& s, int buf, int kq, int r0, int c0, StepOps<C>& o) {
#pragma unroll
  for (int q = 0; q < C::SM; ++q) {
    o.ar[q] = s.a[buf][0][kq][r0 + q * 16];
    o.ai[q] = s.a[buf][1][kq][r0 + q * 16];
  }
#pragma unroll
  for (int q = 0; q < C::SN; ++q) {
    o.br[q] = s.b[buf][0][kq][c0 + q * 16];
    o.bi[q] = s.b[buf][1][kq][c0 + q * 16];
  }
}

// Three real MFMAs per sub-tile and k step (see TileAcc); all 3 SM SN of a step are
// independent, so dependent MFMAs are a full step apart.
template <typename C, bool FULL>
__device__ inline void step_mfma(const StepOps<C>& o, const bool (&rv)[C::SM], const bool (&cv)[C::SN],
                                 TileAcc<C>& acc) {
  typedef typename C::T T;
  constexpr int SM = C::SM, SN = C::SN;
  T as[SM], bs[SN];
#pragma unroll
  for (int q = 0; q < SM; ++q) as[q] = o.ar[q] + o.ai[q];
#pragma unroll
  for (int q = 0; q < SN; ++q) bs[q] = o.br[q] + o.bi[q];
#pragma unroll
  for (int ri = 0; ri < SM; ++ri)
#pragma unroll
    for (int ci = 0; ci < SN; ++ci) {
      if (!FULL && !(rv[ri] && cv[ci])) continue;
      acc.re[ri][ci] = mfma16(o.ar[ri], o.br[ci], acc.re[ri][ci]);
      acc.x[ri][ci] = mfma16(o.ai[ri], o.bi[ci], acc.x[ri][ci]);
      acc.im[ri][ci] = mfma16(as[ri], bs[ci], acc.im[ri][ci]);
    }
}

// One 16-deep slab: the operands of step k+1 are read from LDS while the MFMAs of step k
// run (two register stages).
template <typename C, bool FULL>
__device__ inline void tile_slab(const TileLds<C>& s, int buf, const bool (&rv)[C::SM], const bool (&cv)[C::SN],
                                 TileAcc<C>& acc) {
  const int lane = threadIdx.x & 63, wave = tile_wave();
  const int r0 = (wave >> 1) * (C::BM / 2) + (lane & 15);
  const int c0 = (wave & 1) * (C::BN / 2) + (lane & 15);
  const int kl = lane >> 4;
  StepOps<C> o[2];
  step_load(s, buf, kl, r0, c0, o[0]);
#pragma unroll
  for (int k4 = 0; k4 < TBK / 4; ++k4) {
    if (k4 + 1 < TBK / 4) step_load(s, buf, (k4 + 1) * 4 + kl, r0, c0, o[(k4 + 1) & 1]);
    step_mfma<C, FULL>(o[k4 & 1], rv, cv, acc);
  }
}

// K loop of one tile.  On entry LDS buffer b0 holds slab 0 of op (stored by the previous
// tile's loop, or by tile_start for the first tile).  While the last slab's MFMAs run,
// slab 0 of `next` (when has_next) is loaded and then stored into the other buffer, so
// the next tile's first loads overlap this tile's tail and epilogue.  Returns the buffer
// that holds it.  Every slab ends with a barrier, after the LDS reads of the slab and the
// store of the following one.
template <typename C, bool FULL>
__device__ inline int tile_kloop(const TileOperands<typename C::T>& op, TileLds<C>& s, const bool (&rv)[C::SM],
                                 const bool (&cv)[C::SN], TileAcc<C>& acc, int b0, bool has_next,
                                 const TileOperands<typename C::T>& next) {
  SlabRegs<C> r;
  SlabSrc<C> p = slab_src<C>(op);
  slab_advance<C>(p, op.lda);
  const int nk = op.K / TBK;
  // after the last slab: the next tile's slab 0, or (no next tile) this tile's again,
  // stored into the idle buffer and never read
  const SlabSrc<C> pn = slab_src<C>(has_next ? next : op);
  const int ldn = has_next ? next.lda : op.lda;
  for (int kb = 0; kb < nk; ++kb) {
    const int buf = (b0 + kb) & 1;
    const bool last = kb + 1 == nk;
    SlabSrc<C> q;
    q.a = last ? pn.a : p.a;
    q.b = last ? pn.b : p.b;
    slab_fetch<C>(q, last ? ldn : op.lda, r);
    slab_advance<C>(p, op.lda);
    __builtin_amdgcn_sched_barrier(0);  // issue the loads before the slab's MFMAs
    tile_slab<C, FULL>(s, buf, rv, cv, acc);
    // the store waits for this slab's loads: keep it after the MFMAs
    __builtin_amdgcn_sched_barrier(0);
    tile_stash(s, buf ^ 1, r);
    __syncthreads();
  }
  return (b0 + nk) & 1;
}

// Load the first tile's slab 0 into LDS buffer 0 (later tiles find theirs where the
// previous tile_mma call left it).
template <typename C>
__device__ inline int tile_start(const TileOperands<typename C::T>& op, TileLds<C>& s) {
  SlabRegs<C> r;
  tile_prime<C>(op, r);
  tile_stash(s, 0, r);
  __syncthreads();
  return 0;
}

// Full K loop for one output tile; acc is zeroed here.  Interior tiles run a copy of the
// loop without the per-sub-tile range checks; every check is wave-uniform.  `buf` is the
// LDS buffer holding slab 0 of op on entry and of next on return (see tile_kloop).  A
// persistent loop calls tile_start for its first tile only.
template <typename C>
__device__ inline void tile_mma(const TileOperands<typename C::T>& op, TileLds<C>& s, TileAcc<C>& acc, int& buf,
                                bool has_next, const TileOperands<typename C::T>& next) {
  typedef typename C::T T;
  constexpr int SM = C::SM, SN = C::SN;
#pragma unroll
  for (int ri = 0; ri < SM; ++ri)
#pragma unroll
    for (int ci = 0; ci < SN; ++ci) {
      acc.re[ri][ci] = typename Vec4<T>::type{0, 0, 0, 0};
      acc.im[ri][ci] = typename Vec4<T>::type{0, 0, 0, 0};
      acc.x[ri][ci] = typename Vec4<T>::type{0, 0, 0, 0};
    }
  const int wave = tile_wave();
  const int wr = wave >> 1, wc = wave & 1;
  bool rv[SM], cv[SN];
#pragma unroll
  for (int q = 0; q < SM; ++q) rv[q] = op.row0 + wr * (C::BM / 2) + q * 16 < op.M;
#pragma unroll
  for (int q = 0; q < SN; ++q) cv[q] = op.col0 + wc * (C::BN / 2) + q * 16 < op.N;
  if (op.row0 + C::BM <= op.M && op.col0 + C::BN <= op.N)
    buf = tile_kloop<C, true>(op, s, rv, cv, acc, buf, has_next, next);
  else
    buf = tile_kloop<C, false>(op, s, rv, cv, acc, buf, has_next, next);
#pragma unroll
  for (int ri = 0; ri < SM; ++ri)
#pragma unroll
    for (int ci = 0; ci < SN; ++ci) {
      const typename Vec4<T>::type p1 = acc.re[ri][ci];
      acc.re[ri][ci] = p1 - acc.x[ri][ci];
      acc.im[ri][ci] = acc.im[ri][ci] - p1 - acc.x[ri][ci];
    }
}

// First row of sub-tile ri of this wave, the row offset of accumulator element v, and
// the column of sub-tile ci held by this lane.
template <typename C>
__device__ inline int acc_row_base(int row0, int ri) {
  return row0 + (tile_wave() >> 1) * (C::BM / 2) + ri * 16;
}
template <typename T> __device__ inline int acc_row_off(int v);
template <> __device__ inline int acc_row_off<float>(int v) { return 4 * ((threadIdx.x & 63) >> 4) + v; }
template <> __device__ inline int acc_row_off<double>(int v) { return ((threadIdx.x & 63) >> 4) + 4 * v; }
// Rows of accumulator elements v = 0..3 are row0 + v * AccRowStep: contiguous for FP32
// (one 16-byte access in a column-major matrix), four apart for FP64.
template <typename T> struct AccRowStep;
template <> struct AccRowStep<float> { static constexpr int value = 1; };
template <> struct AccRowStep<double> { static constexpr int value = 4; };
template <typename T>
__device__ inline typename Vec4<T>::type acc_load(const T* p);
template <>
__device__ inline f4v acc_load<float>(const float* p) { return *reinterpret_cast<const f4v*>(p); }
template <>
__device__ inline d4v acc_load<double>(const double* p) { return d4v{p[0], p[4], p[8], p[12]}; }
template <typename T>
__device__ inline void acc_store(T* p, typename Vec4<T>::type v);
template <>
__device__ inline void acc_store<float>(float* p, f4v v) { *reinterpret_cast<f4v*>(p) = v; }
template <>
__device__ inline void acc_store<double>(double* p, d4v v) { p[0] = v[0]; p[4] = v[1]; p[8] = v[2]; p[12] = v[3]; }

template <typename C>
__device__ inline int acc_col(int col0, int ci) {
  return col0 + (tile_wave() & 1) * (C::BN / 2) + ci * 16 + (threadIdx.x & 15);
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
