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
// Operands are staged through LDS in 16-deep slabs.  FP32 tiles load them straight into
// LDS (global_load_lds) through a ring of three stages, two slabs ahead of the MFMAs;
// FP64 tiles load the next slab into registers while the current one feeds the MFMAs
// and store it into the other half of a double buffer.  In a persistent loop the next
// tile's first slab(s) load during the current tile's last one(s).
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

// State of a work-group's tile pipeline between tile products: the LDS stage that holds
// (or will hold) slab 0 of the next product, and how many of its slabs are already being
// loaded.
struct TilePipe {
  int stage, pre;
};

// Register-staged path (FP64): load the first tile's slab 0 into LDS buffer 0 (later
// tiles find theirs where the previous tile_mma call left it).
template <typename C>
__device__ inline TilePipe tile_start(const TileOperands<typename C::T>& op, TileLds<C>& s) {
  SlabRegs<C> r;
  tile_prime<C>(op, r);
  tile_stash(s, 0, r);
  __syncthreads();
  return TilePipe{0, 1};
}

template <typename C>
__device__ inline void tile_zero(TileAcc<C>& acc) {
#pragma unroll
  for (int ri = 0; ri < C::SM; ++ri)
#pragma unroll
    for (int ci = 0; ci < C::SN; ++ci) {
      acc.re[ri][ci] = typename Vec4<typename C::T>::type{0, 0, 0, 0};
      acc.im[ri][ci] = typename Vec4<typename C::T>::type{0, 0, 0, 0};
      acc.x[ri][ci] = typename Vec4<typename C::T>::type{0, 0, 0, 0};
    }
}

// Sub-tile validity of this wave (wave-uniform) and whether the whole tile is interior.
template <typename C>
__device__ inline bool tile_ranges(const TileOperands<typename C::T>& op, bool (&rv)[C::SM], bool (&cv)[C::SN]) {
  const int wave = tile_wave();
  const int wr = wave >> 1, wc = wave & 1;
#pragma unroll
  for (int q = 0; q < C::SM; ++q) rv[q] = op.row0 + wr * (C::BM / 2) + q * 16 < op.M;
#pragma unroll
  for (int q = 0; q < C::SN; ++q) cv[q] = op.col0 + wc * (C::BN / 2) + q * 16 < op.N;
  return op.row0 + C::BM <= op.M && op.col0 + C::BN <= op.N;
}

// Gauss's 3M combination of the three real products (see TileAcc).
template <typename C>
__device__ inline void tile_finish(TileAcc<C>& acc) {
#pragma unroll
  for (int ri = 0; ri < C::SM; ++ri)
#pragma unroll
    for (int ci = 0; ci < C::SN; ++ci) {
      const typename Vec4<typename C::T>::type p1 = acc.re[ri][ci];
      acc.re[ri][ci] = p1 - acc.x[ri][ci];
      acc.im[ri][ci] = acc.im[ri][ci] - p1 - acc.x[ri][ci];
    }
}

// Full K loop for one output tile; acc is zeroed here.  Interior tiles run a copy of the
// loop without the per-sub-tile range checks; every check is wave-uniform.  The pipe
// state carries slab 0 of op in and of next out (see tile_kloop).  A persistent loop
// calls tile_start for its first tile only.
template <typename C>
__device__ inline void tile_mma(const TileOperands<typename C::T>& op, TileLds<C>& s, TileAcc<C>& acc,
                                TilePipe& tp, bool has_next, const TileOperands<typename C::T>& next) {
  tile_zero<C>(acc);
  bool rv[C::SM], cv[C::SN];
  if (tile_ranges<C>(op, rv, cv))
    tp.stage = tile_kloop<C, true>(op, s, rv, cv, acc, tp.stage, has_next, next);
  else
    tp.stage = tile_kloop<C, false>(op, s, rv, cv, acc, tp.stage, has_next, next);
  tile_finish<C>(acc);
}

// ---------------------------------------------------------------------------------------
// FP32 path: operands go from global memory straight into LDS (global_load_lds_dwordx4,
// no registers, no LDS store instructions) through a ring of DLS stages, with slab kb + 2
// in flight while slab kb is multiplied.  A wave's load instruction writes 64 lanes x 16
// bytes contiguously, so each stage is laid out in 1 KB chunks:
//  A [plane][k][BM]: a chunk holds KPC whole k rows; the row quads of k row k are stored
//    XOR-permuted by ((k / 4) % 4) * 4 (bits 2-3 of the quad index);
//  B [plane][col][16 k]: a chunk holds 16 columns; the k quads of column c are stored
//    XOR-permuted by (c / 2) % 4.
// The k index of MFMA step k4 for lane group kl = lane / 16 is 4 kl + k4 (any assignment
// of the 16 k of a slab to (k4, kl) sums the same products), so a lane's four B values of
// a slab are one 16-byte LDS read, and every LDS read below is free of bank conflicts.
constexpr int DLS = 3;

template <typename C>
struct DlShape {
  static constexpr int QPR = C::BM / 4;       // row quads per k row of A
  static constexpr int KPC = 64 / QPR;        // k rows per A chunk
  static constexpr int ACH = 2 * TBK / KPC;   // A chunks per stage (both planes)
  static constexpr int BCH = 2 * C::BN / 16;  // B chunks per stage (16 columns each)
  static constexpr int AW = ACH / 4, BW = BCH / 4;
  static constexpr int NL = AW + BW;          // load instructions per wave per slab
  static_assert(C::BM >= 64 && 64 % QPR == 0 && ACH % 4 == 0 && BCH % 4 == 0, "direct-to-LDS mapping");
};

template <typename C>
struct alignas(16) DlLds {
  float a[DLS][2][TBK][C::BM];
  float b[DLS][2][C::BN][TBK];
};

// This lane's source address of each of its wave's chunks, at slab 0 of one product.
template <typename C>
struct DlSrc {
  const float* a[DlShape<C>::AW];
  const float* b[DlShape<C>::BW];
};

template <typename C>
__device__ inline DlSrc<C> dl_src(const TileOperands<float>& op) {
  typedef DlShape<C> S;
  const int lane = threadIdx.x & 63, w = tile_wave();
  DlSrc<C> p;
#pragma unroll
  for (int i = 0; i < S::AW; ++i) {
    const int c = w * S::AW + i, plane = c / (S::ACH / 2);
    const int k = (c % (S::ACH / 2)) * S::KPC + lane / S::QPR;
    const int quad = (lane % S::QPR) ^ (((k >> 2) & 3) << 2);
    int row = op.row0 + 4 * quad;
    row = row < op.M ? row : op.M - 4;
    p.a[i] = op.A + plane * op.a_ps + (long long)k * op.lda + row;
  }
#pragma unroll
  for (int i = 0; i < S::BW; ++i) {
    const int c = w * S::BW + i, plane = c / (S::BCH / 2);
    const int col = (c % (S::BCH / 2)) * 16 + lane / 4;
    const int kq = (lane & 3) ^ ((col >> 1) & 3);
    int gc = op.col0 + col;
    gc = gc < op.N ? gc : op.N - 1;
    p.b[i] = op.B + plane * op.b_ps + (long long)gc * op.ldb + 4 * kq;
  }
  return p;
}

// One global_load_lds_dwordx4: every lane's 16 bytes at src land at dst + 16 * lane (dst
// wave-uniform).
__device__ inline void lds_dma16(const float* src, float* dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
}

// Start loading slab `slab` of a product (sources p, leading dimension lda) into a stage.
template <typename C>
__device__ inline void dl_issue(const DlSrc<C>& p, int slab, int lda, DlLds<C>& s, int stage) {
  typedef DlShape<C> S;
  const int w = tile_wave();
  const long long ka = (long long)slab * TBK * lda;
#pragma unroll
  for (int i = 0; i < S::AW; ++i) {
    const int c = w * S::AW + i, plane = c / (S::ACH / 2);
    float* dst = &s.a[stage][plane][(c % (S::ACH / 2)) * S::KPC][0];
    lds_dma16(p.a[i] + ka, dst);
  }
#pragma unroll
  for (int i = 0; i < S::BW; ++i) {
    const int c = w * S::BW + i, plane = c / (S::BCH / 2);
    float* dst = &s.b[stage][plane][(c % (S::BCH / 2)) * 16][0];
    lds_dma16(p.b[i] + slab * TBK, dst);
  }
}

// Wait until at most n slabs of this wave's loads are still in flight (n <= 2).
// s_waitcnt operand that waits for vmcnt <= v only: vmcnt bits 3:0 and 15:14, expcnt
// (7: no wait) bits 6:4, lgkmcnt (15: no wait) bits 11:8.
constexpr int vmcnt_only(int v) { return (v & 15) | ((v >> 4) << 14) | 0x0F70; }

template <typename C>
__device__ inline void dl_wait(int n) {
  constexpr int NL = DlShape<C>::NL;
  static_assert(2 * NL < 64, "vmcnt field");
  if (n >= 2)
    __builtin_amdgcn_s_waitcnt(vmcnt_only(2 * NL));
  else if (n == 1)
    __builtin_amdgcn_s_waitcnt(vmcnt_only(NL));
  else
    __builtin_amdgcn_s_waitcnt(vmcnt_only(0));
}

// One slab of a wave whose first NR sub-tile rows and NC sub-tile columns lie inside the
// product (compile-time counts: edge tiles run straight-line code for exactly their valid
// sub-tiles).
template <typename C, int NR, int NC>
__device__ inline void dl_slab(const DlLds<C>& s, int st, TileAcc<C>& acc) {
  const int lane = threadIdx.x & 63, wave = tile_wave();
  const int rl = lane & 15, kl = lane >> 4;
  const int wr = wave >> 1, wc = wave & 1;
  f4v br[NC > 0 ? NC : 1], bi[NC > 0 ? NC : 1];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int col = wc * (C::BN / 2) + q * 16 + rl;
    const int off = col * TBK + 4 * (kl ^ ((col >> 1) & 3));
    br[q] = *static_cast<const f4v*>(__builtin_assume_aligned(&s.b[st][0][0][0] + off, 16));
    bi[q] = *static_cast<const f4v*>(__builtin_assume_aligned(&s.b[st][1][0][0] + off, 16));
  }
  int aoff[NR > 0 ? NR : 1];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int row = wr * (C::BM / 2) + q * 16 + rl;
    aoff[q] = 4 * ((row >> 2) ^ (kl << 2)) + (row & 3);
  }
#pragma unroll
  for (int k4 = 0; k4 < TBK / 4; ++k4) {
    const int k = 4 * kl + k4;
    float ar[NR > 0 ? NR : 1], ai[NR > 0 ? NR : 1], as[NR > 0 ? NR : 1], bs[NC > 0 ? NC : 1];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      ar[q] = s.a[st][0][k][aoff[q]];
      ai[q] = s.a[st][1][k][aoff[q]];
      as[q] = ar[q] + ai[q];
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) bs[q] = br[q][k4] + bi[q][k4];
#pragma unroll
    for (int ri = 0; ri < NR; ++ri)
#pragma unroll
      for (int ci = 0; ci < NC; ++ci) {
        acc.re[ri][ci] = mfma16(ar[ri], br[ci][k4], acc.re[ri][ci]);
        acc.x[ri][ci] = mfma16(ai[ri], bi[ci][k4], acc.x[ri][ci]);
        acc.im[ri][ci] = mfma16(as[ri], bs[ci], acc.im[ri][ci]);
      }
  }
}

// K loop of one product.  Slabs form one stream across the products of a work-group:
// position p < nk is slab p of op, position nk + i slab i of next.  Before slab kb is
// used, positions kb and kb + 1 have been issued; after the barrier that follows its
// arrival, position kb + 2 is issued into the stage that slab kb - 1 used.
template <typename C, int NR, int NC>
__device__ inline void dl_kloop(const TileOperands<float>& op, DlLds<C>& s, TileAcc<C>& acc, TilePipe& tp,
                                bool has_next, const TileOperands<float>& next) {
  const int nk = op.K / TBK;
  const int nkn = has_next ? next.K / TBK : 0;
  const DlSrc<C> p = dl_src<C>(op);
  const DlSrc<C> pn = dl_src<C>(next);  // next is a valid product even when !has_next
  int npos = tp.pre;                     // positions issued so far
#pragma unroll
  for (int pos = 0; pos < 2; ++pos) {
    if (npos != pos) continue;
    if (pos < nk) {
      dl_issue<C>(p, pos, op.lda, s, (tp.stage + pos) % DLS);
      npos = pos + 1;
    } else if (pos - nk < nkn) {
      dl_issue<C>(pn, pos - nk, next.lda, s, (tp.stage + pos) % DLS);
      npos = pos + 1;
    }
  }
  for (int kb = 0; kb < nk; ++kb) {
    dl_wait<C>(npos - 1 - kb);
    __builtin_amdgcn_s_barrier();
    if (npos == kb + 2) {
      const int pos = kb + 2;
      if (pos < nk) {
        dl_issue<C>(p, pos, op.lda, s, (tp.stage + pos) % DLS);
        npos = pos + 1;
      } else if (pos - nk < nkn) {
        dl_issue<C>(pn, pos - nk, next.lda, s, (tp.stage + pos) % DLS);
        npos = pos + 1;
      }
    }
    dl_slab<C, NR, NC>(s, (tp.stage + kb) % DLS, acc);
  }
  tp.stage = (tp.stage + nk) % DLS;
  tp.pre = npos - nk > 0 ? npos - nk : 0;
}

template <typename C>
__device__ inline TilePipe tile_start(const TileOperands<float>&, DlLds<C>&) {
  return TilePipe{0, 0};
}

// Picks the K loop compiled for this wave's valid sub-tile counts (nr <= NR, nc <= NC).
template <typename C, int NR, int NC>
__device__ inline void dl_run(int nr, int nc, const TileOperands<float>& op, DlLds<C>& s, TileAcc<C>& acc,
                              TilePipe& tp, bool has_next, const TileOperands<float>& next) {
  if constexpr (NR > 0) {
    if (nr < NR) {
      dl_run<C, NR - 1, NC>(nr, nc, op, s, acc, tp, has_next, next);
      return;
    }
  }
  if constexpr (NC > 0) {
    if (nc < NC) {
      dl_run<C, NR, NC - 1>(nr, nc, op, s, acc, tp, has_next, next);
      return;
    }
  }
  dl_kloop<C, NR, NC>(op, s, acc, tp, has_next, next);
}

template <typename C>
__device__ inline void tile_mma(const TileOperands<float>& op, DlLds<C>& s, TileAcc<C>& acc, TilePipe& tp,
                                bool has_next, const TileOperands<float>& next) {
  tile_zero<C>(acc);
  bool rv[C::SM], cv[C::SN];
  tile_ranges<C>(op, rv, cv);
  int nr = 0, nc = 0;  // valid sub-tiles come first along each direction
#pragma unroll
  for (int q = 0; q < C::SM; ++q) nr += rv[q];
#pragma unroll
  for (int q = 0; q < C::SN; ++q) nc += cv[q];
  dl_run<C, C::SM, C::SN>(nr, nc, op, s, acc, tp, has_next, next);
  tile_finish<C>(acc);
}

// The LDS of a work-group's tile pipeline: the direct-to-LDS ring for FP32, the
// register-staged double buffer for FP64.
template <typename C, typename T = typename C::T>
struct TileSmemSel {
  typedef TileLds<C> type;
};
template <typename C>
struct TileSmemSel<C, float> {
  typedef DlLds<C> type;
};
template <typename C>
using TileSmem = typename TileSmemSel<C>::type;

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
__device__ inline f4v acc_load<float>(const float* p) { return ld_global<f4v>(p); }
template <>
__device__ inline d4v acc_load<double>(const double* p) {
  return d4v{ld_global<double>(p), ld_global<double>(p + 4), ld_global<double>(p + 8), ld_global<double>(p + 12)};
}
template <typename T>
__device__ inline void acc_store(T* p, typename Vec4<T>::type v);
template <>
__device__ inline void acc_store<float>(float* p, f4v v) { *(__attribute__((address_space(1))) f4v*)p = v; }
template <>
__device__ inline void acc_store<double>(double* p, d4v v) {
  __attribute__((address_space(1))) double* g = (__attribute__((address_space(1))) double*)p;
  g[0] = v[0];
  g[4] = v[1];
  g[8] = v[2];
  g[12] = v[3];
}

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
