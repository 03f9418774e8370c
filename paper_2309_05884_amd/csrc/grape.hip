// GRAPE hot path on gfx950: slice propagators, forward/backward sweeps, objective and
// exact gradient (Eqs. (3)-(4); App. B, Eq. (B2) to all orders).
//
// Per block theta and slice j (an "entry"):
//   X_j = -i dt (H0 + sum_k u[j,k] H_k)                                (Eq. (3))
//   ||X_j||_1 in FP64 picks (q_j, s_j): Taylor degree p = q_j * r and s_j squarings,
//   the cheapest pair with ||X_j||_1 / 2^s_j <= theta_p (truncated-Taylor backward
//   error below the unit roundoff of the working precision);
//   Y = X_j / 2^s_j;  T = T_p(Y) by Paterson-Stockmeyer (powers Y^2..Y^r, then q_j-1
//   Horner products in Y^r);  U_j = T^(2^s_j).
// All products are complex GEMMs on the matrix cores (FP64 or FP32 MFMA).
// Sweeps: psi_{j+1} = U_j psi_j (forward), lambda_j = U_j^dag lambda_{j+1} (backward),
// one work-group per block with the state in LDS.  Objective o = <psi_f|psi_N> in FP64.
// Gradient: do/du[j,k] = <lambda_{j+1}| L(X_j, -i dt H_k) |psi_j>, with L the Frechet
// derivative of exp, evaluated through the vector series
//   L(Y,E) = sum_{i,t} i! t!/(i+t+1)! (Y^dag)^i ... : <b_i|E|a_t>, a_t = Y^t psi/t!,
//   b_i = (-Y)^i lambda/i!,
// over R sub-steps when ||X|| is large; the products H_o [vectors of all slices] are
// GEMMs with the block operators shared by every slice, and the inner products are
// accumulated in FP64.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "mfma_tile.h"
#include "qoc_internal.h"
#include "taylor_table.h"

namespace qoc {

// ===================================================================== plan structures
struct JobDev {
  int m, mp, d, pad_;
  long long h_off;       // operator planes of this block in the system buffer (elements)
  long long ent_off;     // first entry index of this job within a segment
  long long item_off;    // first expm GEMM item of this job
  long long ebuf_off;    // expm buffers of this job (elements of T)
  long long psi_off;     // forward states (elements of T), planes of mp x (N+1)d
  long long lam_off;     // costates (elements of T), planes of mp x N d
  long long gbase_off;   // gradient slots (elements of T)
  long long gslot;       // elements per gradient slot (2 planes x mp x CC)
  long long gacc_off;    // gradient accumulators (complex FP64 entries)
  long long state_off;   // block offset in the caller's panels (complex entries)
  int tiles;             // ceil(mp / 64)
  int cc;                // gradient columns per chunk (multiple of 16)
};

struct PanelDesc {       // one panel GEMM entry: Z_o = H_o * V for job J
  int job, op;
  long long item_off;
  int tiles_m, tiles_n;
};

}  // namespace qoc

struct qoc_plan_s {
  qoc_system_s* sys = nullptr;
  int prec = 0;
  int N = 0, K = 0;
  double dt = 0.0, u_bound = 0.0;
  int r = 4, qmax = 4, smax = 0;
  double norm_bound = 0.0;
  int seg_len = 0, nseg = 0;
  int R = 1, Q = 1;
  int chunk = 0;  // slices per gradient chunk
  int nslots = 0;
  size_t elem = 8;
  // workspace layout (bytes)
  size_t off_flags = 0, off_ent = 0, off_T = 0, bytes = 0;
  size_t ent_stride_T = 0;
  long long expm_items = 0, panel_items = 0;
  int entries_per_seg = 0;
  int max_mpd = 0;
  size_t off_gacc = 0;
  size_t sweep_lds_elems = 0;
  int max_cc = 0;
  std::vector<qoc::JobDev> jobs;
  std::vector<qoc::PanelDesc> panels;
  qoc::DeviceBuffer d_jobs, d_panels;
  qoc::DeviceBuffer d_theta, d_w;
  int grid_gemm = 512;
};

namespace qoc {

// ===================================================================== small helpers
__device__ inline double warp_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T>
__device__ inline T* tplane(char* ws, size_t off_T, long long elem_off) {
  return reinterpret_cast<T*>(ws + off_T) + elem_off;
}

// ===================================================================== generator + norm
// 1-norm of H0 + sum_k u_k H_k (FP64): one wave per column, lanes over rows (coalesced),
// then the largest column sum over the work-group.  red: 256 doubles of LDS.
__device__ inline double block_col_norm(const double* H, size_t plane, int mp, int m, int K, const double* uj,
                                        double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double cmax = 0.0;
  for (int c = wave; c < m; c += nw) {
    double cs = 0.0;
    for (int rr = lane; rr < m; rr += 64) {
      const size_t idx = (size_t)rr + (size_t)c * mp;
      double hr = 0.0, hi = 0.0;
      for (int o = 0; o <= K; ++o) {
        hr += uj[o] * H[(size_t)(2 * o) * plane + idx];
        hi += uj[o] * H[(size_t)(2 * o + 1) * plane + idx];
      }
      cs += hypot(hr, hi);
    }
    cs = warp_sum(cs);
    cmax = fmax(cmax, cs);
  }
  red[threadIdx.x] = cmax;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const double v = red[0];
  __syncthreads();
  return v;
}

// One work-group per entry (job, slice of the segment).  Pass 1: FP64 column sums of
// |H_j| (exact 1-norm), Pass 2: Y = -i dt 2^-s H_j in the working precision.
template <typename T>
__global__ void __launch_bounds__(256) k_generator(const JobDev* jobs, int njobs, const double* H64, const double* u,
                                                   int K, double dt, int seg_j0, int seg_len, int N, char* ws,
                                                   size_t off_T, int* ent_s, int* ent_q, double* ent_norm, int* flags,
                                                   const double* theta, int r, int qmax, int smax, double norm_bound) {
  __shared__ double red[256];
  __shared__ int sq[2];
  const int e = blockIdx.x;
  int J = 0;
  while (J + 1 < njobs && jobs[J + 1].ent_off <= e) ++J;
  const JobDev jb = jobs[J];
  const int jl = e - (int)jb.ent_off;
  if (jl >= seg_len) return;
  const int j = seg_j0 + jl;
  const int m = jb.m, mp = jb.mp;
  const size_t plane = (size_t)mp * mp;
  const double* H = H64 + jb.h_off;
  double uj[17];
  bool finite = true;
  uj[0] = 1.0;
  for (int k = 0; k < K; ++k) {
    uj[k + 1] = u[(size_t)j * K + k];
    finite = finite && isfinite(uj[k + 1]);
  }
  const double cmax = block_col_norm(H, plane, mp, m, K, uj, red);
  if (threadIdx.x == 0) {
    double nx = dt * cmax;
    int flag = 0;
    if (!finite || !isfinite(nx)) flag |= 2;
    if (nx > norm_bound * (1.0 + 1e-12)) flag |= 1;
    int best_q = qmax, best_s = 0, best_cost = 1 << 30;
    for (int q = qmax; q >= 1; --q) {
      double th = theta[q * r];
      int s = 0;
      while (s < 62 && nx > ldexp(th, s)) ++s;
      int cost = (q - 1) + s;
      if (cost < best_cost) { best_cost = cost; best_q = q; best_s = s; }
    }
    if (best_s > smax) { flag |= 1; best_s = smax; }
    if (flag) atomicOr(flags, flag);
    atomicMax(flags + 1, best_s);
    ent_s[e] = best_s;
    ent_q[e] = best_q;
    ent_norm[e] = nx;
    sq[0] = best_s;
  }
  __syncthreads();
  const double scale = ldexp(dt, -sq[0]);
  const size_t ent_stride = (size_t)(r + 3) * 2 * plane;
  T* Yre = tplane<T>(ws, off_T, jb.ebuf_off) + (size_t)jl * ent_stride;
  T* Yim = Yre + plane;
  for (size_t idx = threadIdx.x; idx < plane; idx += blockDim.x) {
    const int rr = (int)(idx % mp), c = (int)(idx / mp);
    double hr = 0.0, hi = 0.0;
    if (rr < m && c < m) {
      for (int o = 0; o <= K; ++o) {
        hr += uj[o] * H[(size_t)(2 * o) * plane + idx];
        hi += uj[o] * H[(size_t)(2 * o + 1) * plane + idx];
      }
    }
    // -i * scale * (hr + i hi) = scale * hi - i scale * hr
    Yre[idx] = (T)(scale * hi);
    Yim[idx] = (T)(-scale * hr);
  }
}

// ===================================================================== expm GEMM steps
enum { STEP_POWER = 0, STEP_HORNER = 1, STEP_SQUARE = 2 };

__constant__ double kInvFact[64];

template <typename T>
__global__ void __launch_bounds__(256) k_expm_step(const JobDev* jobs, int njobs, long long total_items, char* ws,
                                                   size_t off_T, const int* ent_s, const int* ent_q, int mode, int step,
                                                   int r, int seg_len) {
  __shared__ TileLds<T> lds;
  const ItemRange rg = xcd_items(total_items);
  for (long long it = rg.begin; it < rg.end; it += rg.step) {
    int J = 0;
    while (J + 1 < njobs && jobs[J + 1].item_off <= it) ++J;
    const JobDev jb = jobs[J];
    const long long local = it - jb.item_off;
    const int t2 = jb.tiles * jb.tiles;
    const int jl = (int)(local / t2);
    if (jl >= seg_len) continue;
    const int tile = (int)(local % t2);
    const int ti = tile / jb.tiles, tj = tile % jb.tiles;
    const int e = (int)jb.ent_off + jl;
    const int se = ent_s[e], qe = ent_q[e];
    int ia, ib, ic;  // buffer indices: 0 = Y, i-1 = Y^i (i <= r), r, r+1 = ping-pong T
    if (mode == STEP_POWER) {
      ia = step - 2; ib = 0; ic = step - 1;
    } else if (mode == STEP_HORNER) {
      if (qe - 1 < step) continue;
      ia = r + ((step - 1) & 1); ib = r - 1; ic = r + (step & 1);
    } else {
      if (se < step) continue;
      const int h = qe - 1 + step - 1;
      ia = r + (h & 1); ib = ia; ic = r + ((h + 1) & 1);
    }
    const bool final_op = (mode == STEP_SQUARE && step == se) || (mode == STEP_HORNER && se == 0 && step == qe - 1);
    const int mp = jb.mp;
    const size_t plane = (size_t)mp * mp;
    T* base = tplane<T>(ws, off_T, jb.ebuf_off) + (size_t)jl * (size_t)(r + 3) * 2 * plane;
    TileOperands<T> op;
    op.A = base + (size_t)ia * 2 * plane;
    op.a_ps = plane;
    op.lda = mp;
    op.B = base + (size_t)ib * 2 * plane;
    op.b_ps = plane;
    op.ldb = mp;
    op.M = mp;
    op.N = mp;
    op.K = mp;
    op.row0 = ti * TBM;
    op.col0 = tj * TBN;
    TileAcc<T> acc;
    tile_mma(op, lds, acc);
    T* C = base + (size_t)ic * 2 * plane;
    // Horner coefficients: T <- T Y^r + sum_{i<r} c_{l r + i} Y^i, l = q - 1 - step
    double coef[8];
    const int lh = qe - 1 - step;
    if (mode == STEP_HORNER)
      for (int i = 0; i < r; ++i) coef[i] = kInvFact[lh * r + i];
#pragma unroll
    for (int ri = 0; ri < 2; ++ri)
#pragma unroll
      for (int ci = 0; ci < 2; ++ci) {
        const int rbase = acc_row_base(op.row0, ri);
        const int col = acc_col(op.col0, ci);
        if (rbase >= mp || col >= mp) continue;
        typename Vec4<T>::type vr = acc.re[ri][ci], vi = acc.im[ri][ci];
        if (mode == STEP_HORNER) {
          for (int i = 1; i < r; ++i) {
            const T* P = base + (size_t)(i - 1) * 2 * plane;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const size_t idx = (size_t)(rbase + acc_row_off<T>(v)) + (size_t)col * mp;
              vr[v] += (T)coef[i] * P[idx];
              vi[v] += (T)coef[i] * P[idx + plane];
            }
          }
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (rbase + acc_row_off<T>(v) == col && col < jb.m) vr[v] += (T)coef[0];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          T* cr = C + (size_t)(rbase + acc_row_off<T>(v)) + (size_t)col * mp;
          cr[0] = vr[v];
          cr[plane] = vi[v];
        }
        if (final_op) {
          // conjugate transpose for the backward sweep: Udag[col][row] = conj(U[row][col])
          T* D = base + (size_t)(r + 2) * 2 * plane;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            T* dr = D + (size_t)col + (size_t)(rbase + acc_row_off<T>(v)) * mp;
            dr[0] = vr[v];
            dr[plane] = -vi[v];
          }
        }
      }
  }
}

// T0 = c_{qr} Y^r + sum_{i<r} c_{(q-1) r + i} Y^i (elementwise), one work-group per entry
template <typename T>
__global__ void __launch_bounds__(256) k_horner_init(const JobDev* jobs, int njobs, char* ws, size_t off_T,
                                                     const int* ent_s, const int* ent_q, int r, int seg_len) {
  const int e = blockIdx.x;
  int J = 0;
  while (J + 1 < njobs && jobs[J + 1].ent_off <= e) ++J;
  const JobDev jb = jobs[J];
  const int jl = e - (int)jb.ent_off;
  if (jl >= seg_len) return;
  const int q = ent_q[e];
  const bool final_op = q == 1 && ent_s[e] == 0;
  const int mp = jb.mp, m = jb.m;
  const size_t plane = (size_t)mp * mp;
  T* base = tplane<T>(ws, off_T, jb.ebuf_off) + (size_t)jl * (size_t)(r + 3) * 2 * plane;
  T* Tout = base + (size_t)r * 2 * plane;
  const T ctop = (T)kInvFact[q * r];
  T c[8];
  for (int i = 0; i < r; ++i) c[i] = (T)kInvFact[(q - 1) * r + i];
  for (size_t idx = threadIdx.x; idx < plane; idx += blockDim.x) {
    const int rr = (int)(idx % mp), cc = (int)(idx / mp);
    T vr = ctop * base[(size_t)(r - 1) * 2 * plane + idx];
    T vi = ctop * base[(size_t)(r - 1) * 2 * plane + plane + idx];
    for (int i = 1; i < r; ++i) {
      vr += c[i] * base[(size_t)(i - 1) * 2 * plane + idx];
      vi += c[i] * base[(size_t)(i - 1) * 2 * plane + plane + idx];
    }
    if (rr == cc && rr < m) vr += c[0];
    Tout[idx] = vr;
    Tout[idx + plane] = vi;
    if (final_op) {
      T* D = base + (size_t)(r + 2) * 2 * plane;
      D[(size_t)cc + (size_t)rr * mp] = vr;
      D[(size_t)cc + (size_t)rr * mp + plane] = -vi;
    }
  }
}

template <typename T>
__device__ inline const T* entry_U(const JobDev& jb, char* ws, size_t off_T, int jl, int r, int s, int q) {
  const size_t plane = (size_t)jb.mp * jb.mp;
  const T* base = tplane<T>(ws, off_T, jb.ebuf_off) + (size_t)jl * (size_t)(r + 3) * 2 * plane;
  return base + (size_t)(r + ((q - 1 + s) & 1)) * 2 * plane;
}

// ===================================================================== state set-up
// psi0 -> forward store column 0, psi_f -> costate column N-1 (planar, working precision)
template <typename T>
__global__ void k_states_in(const JobDev* jobs, int njobs, const double2* psi0, const double2* psif, char* ws,
                            size_t off_T, int N, int* flags) {
  const int J = blockIdx.y;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  const long long ncol_psi = (long long)(N + 1) * jb.d, ncol_lam = (long long)N * jb.d;
  T* P = tplane<T>(ws, off_T, jb.psi_off);
  T* Lm = tplane<T>(ws, off_T, jb.lam_off);
  const size_t pps = (size_t)jb.mp * ncol_psi, lps = (size_t)jb.mp * ncol_lam;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < jb.mp * jb.d; idx += gridDim.x * blockDim.x) {
    const int c = idx / jb.mp, i = idx % jb.mp;
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    if (i < jb.m) {
      a = psi0[jb.state_off + (long long)c * jb.m + i];
      b = psif[jb.state_off + (long long)c * jb.m + i];
      if (!isfinite(a.x) || !isfinite(a.y) || !isfinite(b.x) || !isfinite(b.y)) atomicOr(flags, 2);
    }
    const size_t cp = (size_t)c * jb.mp + i;                      // column c of the forward store
    const size_t cl = ((size_t)(N - 1) * jb.d + c) * jb.mp + i;   // column (N-1)d + c of the costates
    P[cp] = (T)a.x;
    P[cp + pps] = (T)a.y;
    Lm[cl] = (T)b.x;
    Lm[cl + lps] = (T)b.y;
  }
}

__global__ void k_zero_ints(int* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ===================================================================== sweeps
// Sweep through one segment, one work-group (16 waves) per block, the state in LDS.
// DIR 0: psi_{j+1} = U_j psi_j from the forward store; DIR 1: lambda_j = U_j^dag
// lambda_{j+1} with the conjugate transpose written by the last product of each slice,
// so both directions read their matrix column by column (coalesced across lanes).
// Wave w covers 64 rows and one of G k-ranges; partial sums meet in LDS.
__host__ __device__ inline int sweep_kgroups(int mp) {
  const int R = (mp + 63) / 64;
  return R >= 16 ? 1 : 16 / R;
}

template <typename T, int DIR>
__global__ void __launch_bounds__(1024) k_sweep(const JobDev* jobs, int njobs, char* ws, size_t off_T,
                                                const int* ent_s, const int* ent_q, int r, int seg_j0, int seg_len,
                                                int N) {
  extern __shared__ char smem_raw[];
  const int J = blockIdx.x;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  const int m = jb.m, mp = jb.mp, d = jb.d;
  const int R = (mp + 63) / 64, G = sweep_kgroups(mp);
  T* sre = reinterpret_cast<T*>(smem_raw);  // state [d][mp]
  T* sim = sre + (size_t)d * mp;
  T* pre = sim + (size_t)d * mp;             // partial sums [G][d][mp]
  T* pim = pre + (size_t)G * d * mp;
  T* S = tplane<T>(ws, off_T, DIR == 0 ? jb.psi_off : jb.lam_off);
  const size_t ncol = DIR == 0 ? (size_t)(N + 1) * d : (size_t)N * d;
  const size_t ps = (size_t)mp * ncol;
  const int col_in = DIR == 0 ? seg_j0 : seg_j0 + seg_len - 1;
  for (int idx = threadIdx.x; idx < mp * d; idx += blockDim.x) {
    const int c = idx / mp, i = idx % mp;
    const size_t g = ((size_t)col_in * d + c) * mp + i;
    sre[idx] = S[g];
    sim[idx] = S[g + ps];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kchunk = (m + G - 1) / G;
  const size_t plane = (size_t)mp * mp;
  for (int it = 0; it < seg_len; ++it) {
    const int jl = DIR == 0 ? it : seg_len - 1 - it;
    const int e = (int)jb.ent_off + jl;
    const T* Ub = tplane<T>(ws, off_T, jb.ebuf_off) + (size_t)jl * (size_t)(r + 3) * 2 * plane;
    const T* U = DIR == 0 ? Ub + (size_t)(r + ((ent_q[e] - 1 + ent_s[e]) & 1)) * 2 * plane
                          : Ub + (size_t)(r + 2) * 2 * plane;
    for (int task = wave; task < R * G; task += 16) {
      const int rg = task % R, kg = task / R;
      const int i = rg * 64 + lane;
      const int k0 = kg * kchunk, k1 = min(m, k0 + kchunk);
      T ar0 = T(0), ai0 = T(0), ar1 = T(0), ai1 = T(0);
      if (i < m) {
        const T* col = U + i;
        int k = k0;
        for (; k + 8 <= k1; k += 8) {
          T ur[8], ui[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            ur[q] = col[(size_t)(k + q) * mp];
            ui[q] = col[(size_t)(k + q) * mp + plane];
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const T p0r = sre[k + q], p0i = sim[k + q];
            ar0 += ur[q] * p0r - ui[q] * p0i;
            ai0 += ur[q] * p0i + ui[q] * p0r;
            if (d > 1) {
              const T p1r = sre[mp + k + q], p1i = sim[mp + k + q];
              ar1 += ur[q] * p1r - ui[q] * p1i;
              ai1 += ur[q] * p1i + ui[q] * p1r;
            }
          }
        }
        for (; k < k1; ++k) {
          const T ur = col[(size_t)k * mp], ui = col[(size_t)k * mp + plane];
          ar0 += ur * sre[k] - ui * sim[k];
          ai0 += ur * sim[k] + ui * sre[k];
          if (d > 1) {
            ar1 += ur * sre[mp + k] - ui * sim[mp + k];
            ai1 += ur * sim[mp + k] + ui * sre[mp + k];
          }
        }
      }
      if (i < mp) {
        pre[((size_t)kg * d) * mp + i] = ar0;
        pim[((size_t)kg * d) * mp + i] = ai0;
        if (d > 1) {
          pre[((size_t)kg * d + 1) * mp + i] = ar1;
          pim[((size_t)kg * d + 1) * mp + i] = ai1;
        }
      }
    }
    __syncthreads();
    const int col_out = DIR == 0 ? seg_j0 + jl + 1 : seg_j0 + jl - 1;
    for (int idx = threadIdx.x; idx < mp * d; idx += blockDim.x) {
      const int c = idx / mp, i = idx % mp;
      T vr = T(0), vi = T(0);
      if (i < m)
        for (int kg = 0; kg < G; ++kg) {
          vr += pre[((size_t)kg * d + c) * mp + i];
          vi += pim[((size_t)kg * d + c) * mp + i];
        }
      sre[idx] = vr;
      sim[idx] = vi;
      if (col_out >= 0) {
        const size_t g = ((size_t)col_out * d + c) * mp + i;
        S[g] = vr;
        S[g + ps] = vi;
      }
    }
    __syncthreads();
  }
}

// ===================================================================== objective
// o = sum <psi_f|psi_N>, ||psi_N||^2, ||psi_f||^2 in FP64 with a fixed-order reduction.
template <typename T>
__global__ void __launch_bounds__(1024) k_overlap(const JobDev* jobs, int njobs, char* ws, size_t off_T, int N,
                                                  const int* flags, double* out) {
  __shared__ double red[4][1024];
  double o_r = 0.0, o_i = 0.0, nn = 0.0, nf = 0.0;
  for (int J = 0; J < njobs; ++J) {
    const JobDev jb = jobs[J];
    const T* P = tplane<T>(ws, off_T, jb.psi_off);
    const T* Lm = tplane<T>(ws, off_T, jb.lam_off);
    const size_t pps = (size_t)jb.mp * (N + 1) * jb.d, lps = (size_t)jb.mp * N * jb.d;
    for (int idx = threadIdx.x; idx < jb.m * jb.d; idx += blockDim.x) {
      const int c = idx / jb.m, i = idx % jb.m;
      const size_t gp = ((size_t)N * jb.d + c) * jb.mp + i;
      const size_t gl = ((size_t)(N - 1) * jb.d + c) * jb.mp + i;
      const double pr = P[gp], pi = P[gp + pps], fr = Lm[gl], fi = Lm[gl + lps];
      o_r += fr * pr + fi * pi;
      o_i += fr * pi - fi * pr;
      nn += pr * pr + pi * pi;
      nf += fr * fr + fi * fi;
    }
  }
  red[0][threadIdx.x] = o_r;
  red[1][threadIdx.x] = o_i;
  red[2][threadIdx.x] = nn;
  red[3][threadIdx.x] = nf;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double orr = red[0][0], oii = red[1][0], nN = red[2][0], nF = red[3][0];
    const double raw = orr * orr + oii * oii;
    out[0] = raw / (nN * nF);
    out[1] = raw;
    out[2] = orr;
    out[3] = oii;
    out[4] = nN;
    out[5] = nF;
    int fl = flags[0];
    if (!isfinite(out[0])) fl |= 2;
    out[6] = (double)flags[1];
    out[7] = (double)fl;
  }
}

// ===================================================================== gradient series
// Z_o = H_o * V for every (job, o); V and Z are gradient slots of the job.
template <typename T>
__global__ void __launch_bounds__(256) k_panel_gemm(const JobDev* jobs, const PanelDesc* descs, int ndesc,
                                                    long long total_items, const T* Hsys, char* ws, size_t off_T,
                                                    int vslot) {
  __shared__ TileLds<T> lds;
  const ItemRange rg = xcd_items(total_items);
  for (long long it = rg.begin; it < rg.end; it += rg.step) {
    int D = 0;
    while (D + 1 < ndesc && descs[D + 1].item_off <= it) ++D;
    const PanelDesc pd = descs[D];
    const JobDev jb = jobs[pd.job];
    const long long local = it - pd.item_off;
    const int ti = (int)(local / pd.tiles_n), tj = (int)(local % pd.tiles_n);
    const int mp = jb.mp;
    const size_t hplane = (size_t)mp * mp;
    const size_t vplane = (size_t)mp * jb.cc;
    T* g = tplane<T>(ws, off_T, jb.gbase_off);
    TileOperands<T> op;
    op.A = Hsys + jb.h_off + (size_t)(2 * pd.op) * hplane;
    op.a_ps = hplane;
    op.lda = mp;
    op.B = g + (size_t)vslot * jb.gslot;
    op.b_ps = vplane;
    op.ldb = mp;
    op.M = mp;
    op.N = jb.cc;
    op.K = mp;
    op.row0 = ti * TBM;
    op.col0 = tj * TBN;
    TileAcc<T> acc;
    tile_mma(op, lds, acc);
    T* C = g + (size_t)pd.op * jb.gslot;
#pragma unroll
    for (int ri = 0; ri < 2; ++ri)
#pragma unroll
      for (int ci = 0; ci < 2; ++ci) {
        const int rbase = acc_row_base(op.row0, ri);
        const int col = acc_col(op.col0, ci);
        if (rbase >= mp || col >= jb.cc) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          T* cr = C + (size_t)(rbase + acc_row_off<T>(v)) + (size_t)col * mp;
          cr[0] = acc.re[ri][ci][v];
          cr[vplane] = acc.im[ri][ci][v];
        }
      }
  }
}

// Load a chunk of forward states (src = 0) or costates (src = 1) into a gradient slot.
template <typename T>
__global__ void k_chunk_load(const JobDev* jobs, int njobs, char* ws, size_t off_T, int src, int slot, int j0,
                             int nslices, int N) {
  const int J = blockIdx.y;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  const int mp = jb.mp, d = jb.d;
  T* g = tplane<T>(ws, off_T, jb.gbase_off) + (size_t)slot * jb.gslot;
  const size_t vplane = (size_t)mp * jb.cc;
  const T* S = tplane<T>(ws, off_T, src == 0 ? jb.psi_off : jb.lam_off);
  const size_t sps = (size_t)mp * (src == 0 ? (size_t)(N + 1) * d : (size_t)N * d);
  const long long total = (long long)mp * jb.cc;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int col = (int)(idx / mp), i = (int)(idx % mp);
    const int jj = col / d, c = col % d;
    T vr = T(0), vi = T(0);
    if (jj < nslices) {
      const size_t gs = ((size_t)(j0 + jj) * d + c) * mp + i;
      vr = S[gs];
      vi = S[gs + sps];
    }
    g[idx] = vr;
    g[idx + vplane] = vi;
  }
}

// next = coef (Z_0 + sum_k u[j,k] Z_k), coef = (sign i) (dt/R) / (t+1); optionally acc += next
template <typename T>
__global__ void k_series_combine(const JobDev* jobs, int njobs, char* ws, size_t off_T, const double* u, int K,
                                 int j0, int nslices, double coef_im, int out_slot, int acc_slot, int zero_acc_first) {
  const int J = blockIdx.y;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  const int mp = jb.mp, d = jb.d;
  T* g = tplane<T>(ws, off_T, jb.gbase_off);
  const size_t vplane = (size_t)mp * jb.cc;
  const long long total = (long long)mp * jb.cc;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int col = (int)(idx / mp);
    const int jj = col / d;
    T sr = g[idx], si = g[idx + vplane];  // Z_0
    if (jj < nslices) {
      for (int k = 1; k <= K; ++k) {
        const T uk = (T)u[(size_t)(j0 + jj) * K + (k - 1)];
        sr += uk * g[(size_t)k * jb.gslot + idx];
        si += uk * g[(size_t)k * jb.gslot + idx + vplane];
      }
    } else {
      sr = si = T(0);
    }
    // (i c) * (sr + i si) = -c si + i c sr
    const T c = (T)coef_im;
    const T nr = -c * si, ni = c * sr;
    T* o = g + (size_t)out_slot * jb.gslot;
    o[idx] = nr;
    o[idx + vplane] = ni;
    if (acc_slot >= 0) {
      T* a = g + (size_t)acc_slot * jb.gslot;
      if (zero_acc_first) {
        a[idx] = nr;
        a[idx + vplane] = ni;
      } else {
        a[idx] += nr;
        a[idx + vplane] += ni;
      }
    }
  }
}

// slot_dst = slot_src (both gradient slots)
template <typename T>
__global__ void k_slot_copy(const JobDev* jobs, int njobs, char* ws, size_t off_T, int dst, int src) {
  const int J = blockIdx.y;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  T* g = tplane<T>(ws, off_T, jb.gbase_off);
  const long long total = 2LL * jb.mp * jb.cc;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x)
    g[(size_t)dst * jb.gslot + idx] = g[(size_t)src * jb.gslot + idx];
}

// G[col][k] += sum_{i <= imax} w_{i,t} <b_i | Z_k>, FP64; one wave per (job, column)
template <typename T>
__global__ void __launch_bounds__(256) k_series_dot(const JobDev* jobs, int njobs, char* ws, size_t off_T,
                                                    size_t off_gacc, int K, int bank_slot, int nb, const double* w,
                                                    int zero_first) {
  const int J = blockIdx.y;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (col >= jb.cc) return;
  const int mp = jb.mp;
  const T* g = tplane<T>(ws, off_T, jb.gbase_off);
  const size_t vplane = (size_t)mp * jb.cc;
  double2* G = reinterpret_cast<double2*>(ws + off_gacc) + jb.gacc_off + (size_t)col * K;
  for (int k = 1; k <= K; ++k) {
    const T* Z = g + (size_t)k * jb.gslot + (size_t)col * mp;
    double ar = 0.0, ai = 0.0;
    for (int i = 0; i < nb; ++i) {
      const T* Bv = g + (size_t)(bank_slot + i) * jb.gslot + (size_t)col * mp;
      double pr = 0.0, pi = 0.0;
      for (int row = lane; row < jb.m; row += 64) {
        const double br = Bv[row], bi = Bv[row + vplane];
        const double zr = Z[row], zi = Z[row + vplane];
        pr += br * zr + bi * zi;
        pi += br * zi - bi * zr;
      }
      ar += w[i] * pr;
      ai += w[i] * pi;
    }
    ar = warp_sum(ar);
    ai = warp_sum(ai);
    if (lane == 0) {
      double2 prev = zero_first ? make_double2(0.0, 0.0) : G[k - 1];
      G[k - 1] = make_double2(prev.x + ar, prev.y + ai);
    }
  }
}

// grad[j][k] = 2 Re(conj(o) (-i dt/R) sum_{jobs,copies} G) / (||psi_N||^2 ||psi_f||^2)
__global__ void k_grad_finish(const JobDev* jobs, int njobs, const char* ws, size_t off_gacc, int K, int j0,
                              int nslices, double dt_over_R, const double* out, double* grad) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nslices * K) return;
  const int jj = idx / K, k = idx % K;
  double sr = 0.0, si = 0.0;
  for (int J = 0; J < njobs; ++J) {
    const JobDev jb = jobs[J];
    const double2* G = reinterpret_cast<const double2*>(ws + off_gacc) + jb.gacc_off;
    for (int c = 0; c < jb.d; ++c) {
      const double2 v = G[(size_t)(jj * jb.d + c) * K + k];
      sr += v.x;
      si += v.y;
    }
  }
  // (-i a)(sr + i si) = a si - i a sr
  const double dr = dt_over_R * si, di = -dt_over_R * sr;
  const double orr = out[2], oii = out[3];
  // Re(conj(o) * d)
  const double re = orr * dr + oii * di;
  grad[(size_t)(j0 + jj) * K + k] = 2.0 * re / (out[4] * out[5]);
}

// interleaved complex128 copy of U_j for qoc_propagate
template <typename T>
__global__ void k_export_U(const JobDev* jobs, int njobs, char* ws, size_t off_T, const int* ent_s, const int* ent_q,
                           int r, int seg_j0, int seg_len, int N, double2* out, const long long* out_off) {
  const int e = blockIdx.y;
  int J = 0;
  while (J + 1 < njobs && jobs[J + 1].ent_off <= e) ++J;
  const JobDev jb = jobs[J];
  const int jl = e - (int)jb.ent_off;
  if (jl >= seg_len) return;
  const T* U = entry_U<T>(jb, ws, off_T, jl, r, ent_s[e], ent_q[e]);
  const size_t plane = (size_t)jb.mp * jb.mp;
  double2* dst = out + out_off[J] + (size_t)(seg_j0 + jl) * jb.m * jb.m;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < (long long)jb.m * jb.m;
       idx += (long long)gridDim.x * blockDim.x) {
    const int rr = (int)(idx % jb.m), cc = (int)(idx / jb.m);
    const size_t s = (size_t)rr + (size_t)cc * jb.mp;
    dst[idx] = make_double2((double)U[s], (double)U[s + plane]);
  }
}

// dst = sum_{i < count} slot[first + i] (fixed order)
template <typename T>
__global__ void k_slot_sum(const JobDev* jobs, int njobs, char* ws, size_t off_T, int dst, int first, int count) {
  const int J = blockIdx.y;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  T* g = tplane<T>(ws, off_T, jb.gbase_off);
  const long long total = 2LL * jb.mp * jb.cc;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    T s = T(0);
    for (int i = 0; i < count; ++i) s += g[(size_t)(first + i) * jb.gslot + idx];
    g[(size_t)dst * jb.gslot + idx] = s;
  }
}

// dst += src
template <typename T>
__global__ void k_slot_axpy(const JobDev* jobs, int njobs, char* ws, size_t off_T, int dst, int src) {
  const int J = blockIdx.y;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  T* g = tplane<T>(ws, off_T, jb.gbase_off);
  const long long total = 2LL * jb.mp * jb.cc;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x)
    g[(size_t)dst * jb.gslot + idx] += g[(size_t)src * jb.gslot + idx];
}

// ===================================================================== profiler
// Opt-in, process-wide launch timing for benchmarks: HIP events from a pre-created
// pool are recorded on the launch stream around each kernel of the hot path.
enum ProfKind {
  PK_GENERATOR = 0, PK_EXPM_GEMM = 1, PK_HORNER_INIT = 2, PK_SWEEP_FWD = 3, PK_SWEEP_BWD = 4,
  PK_OVERLAP = 5, PK_GRAD_GEMM = 6, PK_GRAD_VECTOR = 7, PK_GRAD_FINISH = 8, PK_OTHER = 9, PK_COUNT = 10
};

struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec { int kind; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::mutex mu;
};
static Profiler g_prof;

template <class F>
static void timed(int kind, hipStream_t st, F&& launch) {
  if (g_prof.on && g_prof.used + 2 <= g_prof.pool.size()) {
    hipEvent_t a = g_prof.pool[g_prof.used++], b = g_prof.pool[g_prof.used++];
    QOC_HIP(hipEventRecord(a, st));
    launch();
    QOC_HIP(hipEventRecord(b, st));
    g_prof.recs.push_back({kind, a, b});
  } else {
    launch();
  }
}

// Norms and (q, s) choice of every slice, without forming the generators.
__global__ void __launch_bounds__(256) k_slice_norms(const JobDev* jobs, int njobs, const double* H64, const double* u,
                                                     int K, double dt, int N, const double* theta, int r, int qmax,
                                                     int* q_out, int* s_out, double* n_out) {
  __shared__ double red[256];
  const int J = blockIdx.y, j = blockIdx.x;
  if (J >= njobs || j >= N) return;
  const JobDev jb = jobs[J];
  const int m = jb.m, mp = jb.mp;
  const size_t plane = (size_t)mp * mp;
  const double* H = H64 + jb.h_off;
  double uj[17];
  uj[0] = 1.0;
  for (int k = 0; k < K; ++k) uj[k + 1] = u[(size_t)j * K + k];
  const double cmax = block_col_norm(H, plane, mp, m, K, uj, red);
  if (threadIdx.x == 0) {
    double nx = dt * cmax;
    int best_q = qmax, best_s = 0, best_cost = 1 << 30;
    for (int q = qmax; q >= 1; --q) {
      int s = 0;
      while (s < 62 && nx > ldexp(theta[q * r], s)) ++s;
      if ((q - 1) + s < best_cost) { best_cost = (q - 1) + s; best_q = q; best_s = s; }
    }
    q_out[(size_t)J * N + j] = best_q;
    s_out[(size_t)J * N + j] = best_s;
    n_out[(size_t)J * N + j] = nx;
  }
}

// ===================================================================== host driver
static double fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

static void upload_factorials() {
  static bool done = false;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  int dev = 0;
  QOC_HIP(hipGetDevice(&dev));
  static std::vector<int> devices_done;
  if (std::find(devices_done.begin(), devices_done.end(), dev) != devices_done.end()) return;
  double h[64];
  for (int i = 0; i < 64; ++i) h[i] = 1.0 / fact(i);
  QOC_HIP(hipMemcpyToSymbol(HIP_SYMBOL(kInvFact), h, sizeof(h)));
  devices_done.push_back(dev);
  (void)done;
}

template <typename T> inline const T* sys_planes(const qoc_plan_s* P);
template <> inline const double* sys_planes<double>(const qoc_plan_s* P) { return P->sys->h64.as<double>(); }
template <> inline const float* sys_planes<float>(const qoc_plan_s* P) { return P->sys->h32.as<float>(); }

template <typename T>
struct Driver {
  static int* ent_s(const qoc_plan_s* P, char* ws) { return reinterpret_cast<int*>(ws + P->off_ent); }
  static int* ent_q(const qoc_plan_s* P, char* ws) { return ent_s(P, ws) + P->entries_per_seg; }
  static double* ent_norm(const qoc_plan_s* P, char* ws) {
    return reinterpret_cast<double*>(ws + P->off_ent + (size_t)8 * P->entries_per_seg);
  }

  static void expm_segment(qoc_plan_s* P, char* ws, const double* u, int seg_j0, int seg_len, hipStream_t st) {
    const int njobs = (int)P->jobs.size();
    const JobDev* dj = P->d_jobs.as<JobDev>();
    int* flags = reinterpret_cast<int*>(ws + P->off_flags);
    const int nent = P->entries_per_seg;
    timed(PK_GENERATOR, st, [&] { hipLaunchKernelGGL(k_generator<T>, dim3(nent), dim3(256), 0, st, dj, njobs, P->sys->h64.as<double>(), u, P->K,
                       P->dt, seg_j0, seg_len, P->N, ws, P->off_T, ent_s(P, ws), ent_q(P, ws), ent_norm(P, ws), flags,
                       P->d_theta.as<double>(), P->r, P->qmax, P->smax, P->norm_bound); });
    QOC_HIP(hipGetLastError());
    const dim3 grid(P->grid_gemm);
    for (int i = 2; i <= P->r; ++i)
      timed(PK_EXPM_GEMM, st, [&] { hipLaunchKernelGGL(k_expm_step<T>, grid, dim3(256), 0, st, dj, njobs, P->expm_items, ws, P->off_T, ent_s(P, ws),
                         ent_q(P, ws), (int)STEP_POWER, i, P->r, seg_len); });
    timed(PK_HORNER_INIT, st, [&] { hipLaunchKernelGGL(k_horner_init<T>, dim3(nent), dim3(256), 0, st, dj, njobs, ws, P->off_T, ent_s(P, ws), ent_q(P, ws),
                       P->r, seg_len); });
    for (int t = 1; t <= P->qmax - 1; ++t)
      timed(PK_EXPM_GEMM, st, [&] { hipLaunchKernelGGL(k_expm_step<T>, grid, dim3(256), 0, st, dj, njobs, P->expm_items, ws, P->off_T, ent_s(P, ws),
                         ent_q(P, ws), (int)STEP_HORNER, t, P->r, seg_len); });
    for (int t = 1; t <= P->smax; ++t)
      timed(PK_EXPM_GEMM, st, [&] { hipLaunchKernelGGL(k_expm_step<T>, grid, dim3(256), 0, st, dj, njobs, P->expm_items, ws, P->off_T, ent_s(P, ws),
                         ent_q(P, ws), (int)STEP_SQUARE, t, P->r, seg_len); });
    QOC_HIP(hipGetLastError());
  }

  static size_t sweep_lds(const qoc_plan_s* P) { return (size_t)P->sweep_lds_elems * sizeof(T); }

  static void propagate(qoc_plan_s* P, const double* u, double2* out, const long long* out_off, char* ws,
                        hipStream_t st) {
    const int njobs = (int)P->jobs.size();
    int* flags = reinterpret_cast<int*>(ws + P->off_flags);
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, flags, 16);  // status ints only
    for (int sg = 0; sg < P->nseg; ++sg) {
      const int j0 = sg * P->seg_len, len = std::min(P->seg_len, P->N - j0);
      expm_segment(P, ws, u, j0, len, st);
      timed(PK_OTHER, st, [&] { hipLaunchKernelGGL(k_export_U<T>, dim3(64, P->entries_per_seg), dim3(256), 0, st, P->d_jobs.as<JobDev>(), njobs,
                         ws, P->off_T, ent_s(P, ws), ent_q(P, ws), P->r, j0, len, P->N, out, out_off); });
      QOC_HIP(hipGetLastError());
    }
  }

  static void run(qoc_plan_s* P, const double* u, const void* psi0, const void* psif, double* out, double* grad,
                  char* ws, hipStream_t st) {
    const int njobs = (int)P->jobs.size();
    const JobDev* dj = P->d_jobs.as<JobDev>();
    int* flags = reinterpret_cast<int*>(ws + P->off_flags);
    const int N = P->N;
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, flags, 16);  // status ints only
    timed(PK_OTHER, st, [&] { hipLaunchKernelGGL(k_states_in<T>, dim3(8, njobs), dim3(256), 0, st, dj, njobs, (const double2*)psi0,
                       (const double2*)psif, ws, P->off_T, N, flags); });
    QOC_HIP(hipGetLastError());
    // forward: propagators of a segment, then the sequential sweep through it
    for (int sg = 0; sg < P->nseg; ++sg) {
      const int j0 = sg * P->seg_len, len = std::min(P->seg_len, N - j0);
      expm_segment(P, ws, u, j0, len, st);
      timed(PK_SWEEP_FWD, st, [&] { hipLaunchKernelGGL((k_sweep<T, 0>), dim3(njobs), dim3(1024), sweep_lds(P), st, dj, njobs, ws, P->off_T,
                         ent_s(P, ws), ent_q(P, ws), P->r, j0, len, N); });
      QOC_HIP(hipGetLastError());
    }
    timed(PK_OVERLAP, st, [&] { hipLaunchKernelGGL(k_overlap<T>, dim3(1), dim3(1024), 0, st, dj, njobs, ws, P->off_T, N, flags, out); });
    QOC_HIP(hipGetLastError());
    // backward: the last segment's propagators are resident; earlier ones are recomputed
    for (int sg = P->nseg - 1; sg >= 0; --sg) {
      const int j0 = sg * P->seg_len, len = std::min(P->seg_len, N - j0);
      if (sg != P->nseg - 1) expm_segment(P, ws, u, j0, len, st);
      timed(PK_SWEEP_BWD, st, [&] { hipLaunchKernelGGL((k_sweep<T, 1>), dim3(njobs), dim3(1024), sweep_lds(P), st, dj, njobs, ws, P->off_T,
                         ent_s(P, ws), ent_q(P, ws), P->r, j0, len, N); });
      QOC_HIP(hipGetLastError());
    }
    gradient(P, u, out, grad, ws, st);
  }

  // Exact gradient by the Frechet series over R sub-steps (see the file header).
  static void gradient(qoc_plan_s* P, const double* u, double* out, double* grad, char* ws, hipStream_t st) {
    const int njobs = (int)P->jobs.size();
    const JobDev* dj = P->d_jobs.as<JobDev>();
    const int N = P->N, K = P->K, R = P->R, Q = P->Q;
    const double dtR = P->dt / R;
    const int slotA0 = K + 1, slotA1 = K + 2, slotS = K + 3, bank0 = K + 4;
    const dim3 eg(64, njobs);
    const T* H = sys_planes<T>(P);
    const PanelDesc* dp = P->d_panels.as<PanelDesc>();
    const int npanel = (int)P->panels.size();
    auto gemm = [&](int vslot) {
      timed(PK_GRAD_GEMM, st, [&] { hipLaunchKernelGGL(k_panel_gemm<T>, dim3(P->grid_gemm), dim3(256), 0, st, dj, dp, npanel, P->panel_items, H, ws,
                         P->off_T, vslot); });
    };
    for (int j0 = 0; j0 < N; j0 += P->chunk) {
      const int ns = std::min(P->chunk, N - j0);
      // b-series, r = R-1 .. 0:  b_0 = lambda^{(r)}, b_{i+1} = +i (dt/R) H_j b_i / (i+1);
      // lambda^{(r-1)} = exp(-Y) lambda^{(r)} = sum_i b_i
      timed(PK_GRAD_VECTOR, st, [&] { hipLaunchKernelGGL(k_chunk_load<T>, eg, dim3(256), 0, st, dj, njobs, ws, P->off_T, 1, bank0 + (R - 1) * Q, j0,
                         ns, N); });
      for (int rr = R - 1; rr >= 0; --rr) {
        const int bank = bank0 + rr * Q;
        for (int i = 0; i + 1 < Q; ++i) {
          gemm(bank + i);
          timed(PK_GRAD_VECTOR, st, [&] { hipLaunchKernelGGL(k_series_combine<T>, eg, dim3(256), 0, st, dj, njobs, ws, P->off_T, u, K, j0, ns,
                             dtR / (i + 1), bank + i + 1, -1, 0); });
        }
        if (rr > 0)
          timed(PK_GRAD_VECTOR, st, [&] { hipLaunchKernelGGL(k_slot_sum<T>, eg, dim3(256), 0, st, dj, njobs, ws, P->off_T, bank - Q, bank, Q); });
      }
      QOC_HIP(hipGetLastError());
      // a-series, r = 0 .. R-1: a_0 = psi^{(r)}, a_{t+1} = -i (dt/R) H_j a_t / (t+1);
      // the dot products take every (i, t) with i + t <= Q - 1
      timed(PK_GRAD_VECTOR, st, [&] { hipLaunchKernelGGL(k_chunk_load<T>, eg, dim3(256), 0, st, dj, njobs, ws, P->off_T, 0, slotA0, j0, ns, N); });
      int cur = slotA0, nxt = slotA1;
      bool first_dot = true;
      for (int rr = 0; rr < R; ++rr) {
        const int bank = bank0 + rr * Q;
        const bool need_next_state = rr + 1 < R;
        if (need_next_state) timed(PK_GRAD_VECTOR, st, [&] { hipLaunchKernelGGL(k_slot_sum<T>, eg, dim3(256), 0, st, dj, njobs, ws, P->off_T, slotS, cur, 1); });
        for (int t = 0; t < Q; ++t) {
          gemm(cur);
          const double* wt = P->d_w.as<double>() + (size_t)t * Q;
          timed(PK_GRAD_VECTOR, st, [&] { hipLaunchKernelGGL(k_series_dot<T>, dim3((P->max_cc + 3) / 4, njobs), dim3(256), 0, st, dj, njobs, ws,
                             P->off_T, P->off_gacc, K, bank, Q - t, wt, first_dot ? 1 : 0); });
          first_dot = false;
          if (t + 1 < Q || need_next_state) {
            timed(PK_GRAD_VECTOR, st, [&] { hipLaunchKernelGGL(k_series_combine<T>, eg, dim3(256), 0, st, dj, njobs, ws, P->off_T, u, K, j0, ns,
                               -dtR / (t + 1), nxt, need_next_state ? slotS : -1, 0); });
            std::swap(cur, nxt);
          }
        }
        // a_0 of the next sub-step is psi^{(r+1)} = sum_t a_t, held in slotS
        if (need_next_state)
          timed(PK_GRAD_VECTOR, st, [&] { hipLaunchKernelGGL(k_slot_sum<T>, eg, dim3(256), 0, st, dj, njobs, ws, P->off_T, cur, slotS, 1); });
      }
      QOC_HIP(hipGetLastError());
      timed(PK_GRAD_FINISH, st, [&] { hipLaunchKernelGGL(k_grad_finish, dim3((ns * K + 255) / 256), dim3(256), 0, st, dj, njobs, ws, P->off_gacc, K, j0,
                         ns, dtR, out, grad); });
      QOC_HIP(hipGetLastError());
    }
  }
};

}  // namespace qoc

using namespace qoc;

extern "C" {

qoc_status qoc_plan_create(qoc_system S, int precision, int N, double dt, double u_bound, size_t max_ws,
                           qoc_plan* out) {
  return guarded([&] {
    QOC_REQUIRE(S && out, QOC_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    QOC_REQUIRE(precision == QOC_C128 || precision == QOC_C64, QOC_ERR_INVALID_ARG, "unknown precision");
    QOC_REQUIRE(N >= 1 && N <= (1 << 24), QOC_ERR_INVALID_ARG, "N must be in 1..2^24");
    QOC_REQUIRE(std::isfinite(dt) && dt > 0.0, QOC_ERR_INVALID_ARG, "dt must be positive and finite");
    QOC_REQUIRE(std::isfinite(u_bound) && u_bound >= 0.0, QOC_ERR_INVALID_ARG, "u_bound must be finite and >= 0");
    upload_factorials();
    auto P = std::make_unique<qoc_plan_s>();
    P->sys = S;
    P->prec = precision;
    P->N = N;
    P->K = S->K;
    P->dt = dt;
    P->u_bound = u_bound;
    const bool f64 = precision == QOC_C128;
    P->elem = f64 ? 8 : 4;
    const double* theta = f64 ? kTaylorTheta64 : kTaylorTheta32;
    P->r = f64 ? 4 : 3;
    P->qmax = f64 ? 6 : 4;  // degrees up to 24 (FP64) / 12 (FP32)
    const double unit = f64 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
    // norm bound by the triangle inequality on the exact block 1-norms
    double nb = 0.0;
    for (auto& b : S->blocks) {
      double v = b.norm1[0];
      for (int k = 1; k <= S->K; ++k) v += u_bound * b.norm1[k];
      nb = std::max(nb, dt * v);
    }
    P->norm_bound = nb;
    {
      // squarings the per-slice choice can pick for any norm in (0, nb]: the choice is
      // piecewise constant between the points theta_{qr} 2^s, so evaluate just above each
      auto choose_s = [&](double nx) {
        int best_s = 0, best_cost = 1 << 30;
        for (int q = P->qmax; q >= 1; --q) {
          int sq = 0;
          while (sq < 62 && nx > std::ldexp(theta[q * P->r], sq)) ++sq;
          if ((q - 1) + sq < best_cost) { best_cost = (q - 1) + sq; best_s = sq; }
        }
        return best_s;
      };
      int smax = choose_s(nb);
      for (int q = 1; q <= P->qmax; ++q)
        for (int sq = 0; sq < 62; ++sq) {
          const double x = std::ldexp(theta[q * P->r], sq);
          if (x >= nb) break;
          smax = std::max(smax, choose_s(std::nextafter(x, 1e300)));
        }
      P->smax = smax;
    }
    QOC_REQUIRE(P->smax <= 40, QOC_ERR_NUMERIC, "dt * ||H|| bound too large");
    // Frechet series: R sub-steps with ||Y||_1 <= 2, Q terms with theta^Q / Q! <= unit / 8
    int R = 1;
    while (nb / R > 2.0) R *= 2;
    const double thg = nb / R;
    int Q = 1;
    double term = 1.0;
    while (Q < 60) {
      term = std::pow(thg, Q) / fact(Q);
      if (term <= unit / 8) break;
      ++Q;
    }
    P->R = R;
    P->Q = std::max(Q, 2);
    // jobs
    int max_mpd = 0, max_mp = 0;
    for (auto& b : S->blocks) {
      max_mpd = std::max(max_mpd, b.mp * b.d);
      max_mp = std::max(max_mp, b.mp);
    }
    P->max_mpd = max_mpd;
    QOC_REQUIRE(max_mp <= 4096, QOC_ERR_UNSUPPORTED, "blocks larger than 4096 are not supported by the sweep kernels");
    size_t lds_elems = 0;
    for (auto& b : S->blocks)
      lds_elems = std::max(lds_elems, (size_t)2 * b.d * b.mp * (1 + sweep_kgroups(b.mp)));
    P->sweep_lds_elems = lds_elems;
    QOC_REQUIRE(lds_elems * P->elem <= 160 * 1024, QOC_ERR_UNSUPPORTED,
                "block panel too large for the LDS-resident sweep");
    const int nslots = S->K + 4 + P->R * P->Q;
    P->nslots = nslots;
    // per-slice bytes: expm buffers + states, per job
    size_t per_slice = 0, fixed = 0;
    for (auto& b : S->blocks) {
      per_slice += (size_t)(P->r + 3) * 2 * b.mp * b.mp * P->elem;
      fixed += (size_t)2 * b.mp * ((size_t)(N + 1) * b.d + (size_t)N * b.d) * P->elem;
    }
    // gradient chunk: columns per job chunk*d rounded to 16, capped at 4096 columns
    int chunk = std::min(N, 2048);
    auto grad_bytes = [&](int ch) {
      size_t g = 0;
      for (auto& b : S->blocks) {
        int cc = (ch * b.d + 15) / 16 * 16;
        g += (size_t)nslots * 2 * b.mp * cc * P->elem + (size_t)cc * S->K * 16;
      }
      return g;
    };
    const size_t budget = max_ws ? max_ws : (size_t)200 << 30;
    while (chunk > 16 && fixed + grad_bytes(chunk) + per_slice > budget) chunk /= 2;
    P->chunk = chunk;
    size_t avail = budget > fixed + grad_bytes(chunk) ? budget - fixed - grad_bytes(chunk) : 0;
    long long seg = (long long)(avail / std::max<size_t>(per_slice, 1));
    QOC_REQUIRE(seg >= 1, QOC_ERR_OUT_OF_MEMORY, "workspace budget below one slice of propagators");
    P->seg_len = (int)std::min<long long>(seg, N);
    P->nseg = (N + P->seg_len - 1) / P->seg_len;
    // layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
      size_t o = off;
      off = (off + bytes + 255) / 256 * 256;
      return o;
    };
    P->off_flags = take(256);
    P->entries_per_seg = P->seg_len * (int)S->blocks.size();
    P->off_ent = take((size_t)P->entries_per_seg * 16);
    P->off_gacc = 0;
    long long tel = 0;  // elements of T
    long long ent_off = 0, item_off = 0, gacc = 0;
    int max_cc = 0;
    for (size_t bi = 0; bi < S->blocks.size(); ++bi) {
      auto& b = S->blocks[bi];
      JobDev j{};
      j.m = b.m;
      j.mp = b.mp;
      j.d = b.d;
      j.h_off = b.h_off;
      j.state_off = b.state_off;
      j.tiles = (b.mp + TBM - 1) / TBM;
      j.ent_off = ent_off;
      ent_off += P->seg_len;
      j.item_off = item_off;
      item_off += (long long)P->seg_len * j.tiles * j.tiles;
      j.ebuf_off = tel;
      tel += (long long)P->seg_len * (P->r + 3) * 2 * b.mp * b.mp;
      j.psi_off = tel;
      tel += 2LL * b.mp * (N + 1) * b.d;
      j.lam_off = tel;
      tel += 2LL * b.mp * N * b.d;
      j.cc = (chunk * b.d + 15) / 16 * 16;
      max_cc = std::max(max_cc, j.cc);
      j.gslot = 2LL * b.mp * j.cc;
      j.gbase_off = tel;
      tel += (long long)nslots * j.gslot;
      j.gacc_off = gacc;
      gacc += (long long)j.cc * S->K;
      P->jobs.push_back(j);
    }
    P->max_cc = max_cc;
    P->expm_items = item_off;
    P->off_T = take((size_t)tel * P->elem);
    P->off_gacc = take((size_t)std::max<long long>(gacc, 1) * 16);
    P->bytes = off;
    // panel GEMM descriptors: (job, op) for op = 0..K
    long long pitems = 0;
    for (size_t J = 0; J < P->jobs.size(); ++J)
      for (int o = 0; o <= S->K; ++o) {
        PanelDesc d{};
        d.job = (int)J;
        d.op = o;
        d.item_off = pitems;
        d.tiles_m = (P->jobs[J].mp + TBM - 1) / TBM;
        d.tiles_n = (P->jobs[J].cc + TBN - 1) / TBN;
        pitems += (long long)d.tiles_m * d.tiles_n;
        P->panels.push_back(d);
      }
    P->panel_items = pitems;
    // device tables (set-up only)
    P->d_jobs.alloc(P->jobs.size() * sizeof(JobDev));
    QOC_HIP(hipMemcpy(P->d_jobs.ptr, P->jobs.data(), P->jobs.size() * sizeof(JobDev), hipMemcpyHostToDevice));
    P->d_panels.alloc(std::max<size_t>(1, P->panels.size()) * sizeof(PanelDesc));
    QOC_HIP(hipMemcpy(P->d_panels.ptr, P->panels.data(), P->panels.size() * sizeof(PanelDesc), hipMemcpyHostToDevice));
    P->d_theta.alloc(31 * sizeof(double));
    QOC_HIP(hipMemcpy(P->d_theta.ptr, theta, 31 * sizeof(double), hipMemcpyHostToDevice));
    std::vector<double> w((size_t)P->Q * P->Q, 0.0);
    for (int t = 0; t < P->Q; ++t)
      for (int i = 0; i + t < P->Q; ++i) w[(size_t)t * P->Q + i] = fact(i) * fact(t) / fact(i + t + 1);
    P->d_w.alloc(w.size() * sizeof(double));
    QOC_HIP(hipMemcpy(P->d_w.ptr, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice));
    // persistent GEMM grid: resident work-groups, a multiple of the 8 XCDs
    int dev = 0, ncu = 256, occ = 2;
    QOC_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    QOC_HIP(hipGetDeviceProperties(&prop, dev));
    ncu = prop.multiProcessorCount;
    if (f64)
      QOC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_expm_step<double>, 256, 0));
    else
      QOC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_expm_step<float>, 256, 0));
    P->grid_gemm = std::max(8, ncu * std::max(1, occ) / 8 * 8);
    // the sweeps keep the state and partial sums in LDS; allow the dynamic size beyond 64 KB
    const int lds = (int)(P->sweep_lds_elems * P->elem);
    if (f64) {
      QOC_HIP(hipFuncSetAttribute((const void*)k_sweep<double, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
      QOC_HIP(hipFuncSetAttribute((const void*)k_sweep<double, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    } else {
      QOC_HIP(hipFuncSetAttribute((const void*)k_sweep<float, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
      QOC_HIP(hipFuncSetAttribute((const void*)k_sweep<float, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    }
    *out = P.release();
  });
}

void qoc_plan_free(qoc_plan p) { delete p; }

qoc_status qoc_plan_workspace_size(qoc_plan P, size_t* bytes) {
  return guarded([&] {
    QOC_REQUIRE(P && bytes, QOC_ERR_INVALID_ARG, "null argument");
    *bytes = P->bytes;
  });
}

qoc_status qoc_plan_info(qoc_plan P, int64_t* info, int cap) {
  return guarded([&] {
    QOC_REQUIRE(P && info, QOC_ERR_INVALID_ARG, "null argument");
    int64_t v[10] = {P->seg_len, P->nseg, P->r, (int64_t)P->qmax * P->r, P->Q, P->R, 0, P->smax, P->chunk,
                     P->grid_gemm};
    size_t per_slice = 0;
    for (auto& j : P->jobs) per_slice += (size_t)(P->r + 3) * 2 * j.mp * j.mp * P->elem;
    v[6] = (int64_t)per_slice;
    for (int i = 0; i < cap && i < 10; ++i) info[i] = v[i];
  });
}

qoc_status qoc_propagate(qoc_plan P, const double* u_dev, void* U_out_dev, void* workspace, size_t ws_bytes,
                         void* stream) {
  return guarded([&] {
    QOC_REQUIRE(P && u_dev && U_out_dev && workspace, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(ws_bytes >= P->bytes, QOC_ERR_OUT_OF_MEMORY, "workspace smaller than the plan requires");
    hipStream_t st = (hipStream_t)stream;
    // output offsets per job (complex entries), kept in the workspace flag page
    std::vector<long long> offs;
    long long o = 0;
    for (auto& j : P->jobs) {
      offs.push_back(o);
      o += (long long)P->N * j.m * j.m;
    }
    QOC_REQUIRE(offs.size() <= 24, QOC_ERR_UNSUPPORTED, "too many blocks for the export table");
    long long* d_offs = reinterpret_cast<long long*>(static_cast<char*>(workspace) + P->off_flags + 64);
    QOC_HIP(hipMemcpyAsync(d_offs, offs.data(), offs.size() * sizeof(long long), hipMemcpyHostToDevice, st));
    if (P->prec == QOC_C128)
      Driver<double>::propagate(P, u_dev, (double2*)U_out_dev, d_offs, (char*)workspace, st);
    else
      Driver<float>::propagate(P, u_dev, (double2*)U_out_dev, d_offs, (char*)workspace, st);
  });
}

qoc_status qoc_fidelity_grad(qoc_plan P, const double* u_dev, const void* psi0_dev, const void* psif_dev,
                             double* out_dev, double* grad_dev, void* workspace, size_t ws_bytes, void* stream) {
  return guarded([&] {
    QOC_REQUIRE(P && u_dev && psi0_dev && psif_dev && out_dev && grad_dev && workspace, QOC_ERR_INVALID_ARG,
                "null argument");
    QOC_REQUIRE(ws_bytes >= P->bytes, QOC_ERR_OUT_OF_MEMORY, "workspace smaller than the plan requires");
    hipStream_t st = (hipStream_t)stream;
    if (P->prec == QOC_C128)
      Driver<double>::run(P, u_dev, psi0_dev, psif_dev, out_dev, grad_dev, (char*)workspace, st);
    else
      Driver<float>::run(P, u_dev, psi0_dev, psif_dev, out_dev, grad_dev, (char*)workspace, st);
  });
}


qoc_status qoc_profile_begin(int max_launches) {
  return guarded([&] {
    QOC_REQUIRE(max_launches >= 0 && max_launches <= (1 << 22), QOC_ERR_INVALID_ARG, "max_launches out of range");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    size_t want = (size_t)2 * max_launches;
    while (g_prof.pool.size() < want) {
      hipEvent_t e;
      QOC_HIP(hipEventCreate(&e));
      g_prof.pool.push_back(e);
    }
    g_prof.used = 0;
    g_prof.recs.clear();
    g_prof.on = true;
  });
}

qoc_status qoc_profile_end(double* ms, int64_t* launches, int cap) {
  return guarded([&] {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = false;
    std::vector<double> acc(PK_COUNT, 0.0);
    std::vector<int64_t> cnt(PK_COUNT, 0);
    for (auto& r : g_prof.recs) {
      QOC_HIP(hipEventSynchronize(r.b));
      float t = 0.f;
      QOC_HIP(hipEventElapsedTime(&t, r.a, r.b));
      acc[r.kind] += t;
      cnt[r.kind] += 1;
    }
    for (int i = 0; i < cap && i < PK_COUNT; ++i) {
      if (ms) ms[i] = acc[i];
      if (launches) launches[i] = cnt[i];
    }
    g_prof.recs.clear();
    g_prof.used = 0;
  });
}

qoc_status qoc_plan_slice_stats(qoc_plan P, const double* u_dev, int32_t* q_host, int32_t* s_host, double* norm_host,
                                void* stream) {
  return guarded([&] {
    QOC_REQUIRE(P && u_dev && q_host && s_host && norm_host, QOC_ERR_INVALID_ARG, "null argument");
    hipStream_t st = (hipStream_t)stream;
    const int njobs = (int)P->jobs.size();
    const size_t cnt = (size_t)njobs * P->N;
    DeviceBuffer q(cnt * 4), sbuf(cnt * 4), nrm(cnt * 8);
    hipLaunchKernelGGL(k_slice_norms, dim3(P->N, njobs), dim3(256), 0, st, P->d_jobs.as<JobDev>(), njobs,
                       P->sys->h64.as<double>(), u_dev, P->K, P->dt, P->N, P->d_theta.as<double>(), P->r, P->qmax,
                       q.as<int>(), sbuf.as<int>(), nrm.as<double>());
    QOC_HIP(hipGetLastError());
    QOC_HIP(hipMemcpyAsync(q_host, q.ptr, cnt * 4, hipMemcpyDeviceToHost, st));
    QOC_HIP(hipMemcpyAsync(s_host, sbuf.ptr, cnt * 4, hipMemcpyDeviceToHost, st));
    QOC_HIP(hipMemcpyAsync(norm_host, nrm.ptr, cnt * 8, hipMemcpyDeviceToHost, st));
    QOC_HIP(hipStreamSynchronize(st));
  });
}

}  // extern "C"
