// GRAPE hot path on gfx950: slice propagators, forward/backward sweeps, objective and
// exact gradient (Eqs. (3)-(4); App. B, Eq. (B2) to all orders), for one problem or a
// batch of independent problems (each its own system, slice count and controls).
//
// Per block theta and slice j (an "entry"):
//   X_j = -i dt (H0 + sum_k u[j,k] H_k)                                (Eq. (3))
//   ||X_j||_1 in FP64 picks (q_j, s_j): Taylor degree p = q_j * r and s_j squarings,
//   the cheapest pair with ||X_j||_1 / 2^s_j <= theta_p (truncated-Taylor backward
//   error below the unit roundoff of the working precision);
//   Y = X_j / 2^s_j;  T = T_p(Y) by Paterson-Stockmeyer (powers Y^2..Y^r, then q_j-1
//   Horner products in Y^r);  U_j = T^(2^s_j).
// All products are complex GEMMs on the matrix cores (FP64 or FP32 MFMA).
// Sweeps: psi_{j+1} = U_j psi_j (forward), lambda_j = U_j^dag lambda_{j+1} (backward,
// as dot products down the columns of the same stored U), sequential in j; a block's rows
// are split over ceil(m / 64) (FP32) or ceil(m / 32) (FP64) work-groups that hand the new
// state to each other after every slice, and a block that fits one work-group keeps its
// state in LDS.  Objective o = <psi_f|psi_N>
// in FP64.
// Gradient: do/du[j,k] = <lambda_{j+1}| L(X_j, -i dt H_k) |psi_j>, with L the Frechet
// derivative of exp, through the vector series
//   <lambda|L(Y,E)|psi> = sum_{i+t<Q} i! t!/(i+t+1)! <b_i|E|a_t>,
//   a_t = Y^t psi / t!,  b_i = (-Y)^i lambda / i!   (Y anti-Hermitian),
// over R sub-steps when ||X|| is large; the products H_o [vectors of all slices] are
// GEMMs with the block operators shared by every slice, and the inner products are
// accumulated in FP64.
//
// A "job" is one (problem, block) pair; jobs of a problem are contiguous.  Slices are
// processed in segments of equal length for every job; a job whose problem has fewer
// slices simply has less (or no) work in the later segments.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <memory>
#include <mutex>
#include <type_traits>

#include "mfma_tile.h"
#include "qoc_internal.h"
#include "taylor12.h"
#include "taylor_table.h"

namespace qoc {

// ===================================================================== plan structures
struct JobDev {
  int m, mp, d, prob;
  int N, K;              // the problem's slices and controls
  int tiles_m, tiles_n;  // propagator GEMM tiles per matrix (rows, columns)
  int cc;                // gradient columns per chunk (multiple of 16)
  double dt;
  const double* h64;     // FP64 operator planes of this block
  const void* hT;        // working-precision operator planes of this block
  const void* pwT;       // working-precision operator products (qoc_system_s::pw*), or null
  long long pw_off;      // ... or their workspace copy (elements of T; -1: none)
  long long ent_off;     // first entry (slice of a segment) of this job
  long long item_off;    // first propagator GEMM item of this job
  long long ubuf_off;    // propagators of the segment: per slice U (elements of T)
  long long uslot;       // elements per propagator slot: U (2 planes), or U and the product
                         // tree's second half (4 planes) when the plan has room for both
  long long sbuf_off;    // Taylor scratch of one chunk: per slice Y..Y^r and two ping-pong buffers
  long long psi_off;     // forward states (elements of T), planes of mp x (N+1)d
  long long lam_off;     // costates (elements of T), planes of mp x N d
  long long gbase_off;   // gradient slots (elements of T)
  long long gslot;       // elements per gradient slot (2 planes x mp x cc)
  long long gacc_off;    // gradient accumulators (complex FP64 entries)
  long long state_off;   // block offset in the batch's concatenated panels (complex entries)
  long long u_off;       // the problem's offset in the concatenated controls / gradients
  long long uout_off;    // offset of this job's propagators in qoc_propagate's output
  long long xchg_off;    // co-operative sweep state exchange (64-bit words, per direction)
};

struct ProbDev {
  int job_begin, job_end;
  int N, K;
  double dt;
  long long u_off;
};

struct PanelDesc {       // one panel GEMM entry: Z_o = H_o * V for job J
  int job, op;
  long long item_off;
  int tiles_m, tiles_n;
};

// largest index i with key_i <= key over an ascending table (job / descriptor lookup)
__device__ inline int find_job_by_ent(const JobDev* jobs, int n, long long key) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].ent_off <= key) lo = mid; else hi = mid - 1;
  }
  return lo;
}
__device__ inline int find_job_by_item(const JobDev* jobs, int n, long long key) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].item_off <= key) lo = mid; else hi = mid - 1;
  }
  return lo;
}
// Item -> job for a work-group that walks increasing item indices: the cached job is
// reused while the item stays in its range, then a short forward scan (bounded) or a
// binary search finds the next one.
struct ItemCursor {
  int J = -1;
  long long beg = 0, end = -1;
};
template <typename Rec>
__device__ inline int cursor_find(const Rec* recs, int n, long long key, ItemCursor& c) {
  if (key >= c.beg && key < c.end) return c.J;
  int J = -1;
  if (c.J >= 0 && key >= c.end) {
    J = c.J;
    for (int k = 0; k < 8 && J + 1 < n && recs[J + 1].item_off <= key; ++k) ++J;
    if (J + 1 < n && recs[J + 1].item_off <= key) J = -1;  // still short: search
  }
  if (J < 0) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (recs[mid].item_off <= key) lo = mid; else hi = mid - 1;
    }
    J = lo;
  }
  c.J = J;
  c.beg = recs[J].item_off;
  c.end = J + 1 < n ? recs[J + 1].item_off : (1LL << 62);
  return J;
}

__device__ inline int find_desc(const PanelDesc* d, int n, long long key) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].item_off <= key) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// A pointer known to address device (global) memory: loads and stores through it take the
// global path instead of the flat one (whose completion the LDS wait counter also tracks).
template <typename T>
__device__ inline T* global_ptr(T* p) {
  return (T*)(__attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ inline const T* global_ptr(const T* p) {
  return (const T*)(const __attribute__((address_space(1))) T*)p;
}

// the operator products of job jb's block: the system's own, or the workspace copy
template <typename T>
__device__ inline const T* job_products(const JobDev& jb, char* ws, size_t off_T) {
  return jb.pw_off >= 0 ? reinterpret_cast<const T*>(ws + off_T) + jb.pw_off : static_cast<const T*>(jb.pwT);
}

// slices of job J inside the segment starting at seg_j0 (<= 0: none)
__device__ inline int job_len(const JobDev& jb, int seg_j0, int seg_len) { return min(seg_len, jb.N - seg_j0); }

}  // namespace qoc

struct qoc_plan_s {
  std::vector<qoc_system_s*> systems;
  int P = 1;
  int prec = 0;
  int Nmax = 0, Kmax = 0;
  double u_bound = 0.0;
  int r = 4, qmax = 4, smax = 0;
  int t12 = 0;  // slices may use the four-product degree-12 evaluation
  // 2 when the generator forms Y^2 and Y^3 from the operator products (no power GEMMs for
  // them), else 0; with r = 3 it then also forms each slice's first Taylor combination
  int pow_free = 0;
  // Products of systems that do not keep their own (too large for the free memory) live in
  // the workspace and are formed at the start of every call: five passes of set-up GEMMs
  // (product_descs), descriptors on the device, pass p = [pw_pass_begin[p], [p + 1]).
  int pw_mode = 0;  // prepare_powers' decision
  bool pw_ws = false;
  qoc::DeviceBuffer d_pwgemm;
  int pw_pass_begin[6] = {0, 0, 0, 0, 0, 0};
  long long pw_pass_items[5] = {0, 0, 0, 0, 0};
  double norm_bound = 0.0;
  int seg_len = 0, nseg = 0;
  int echunk = 0;  // slices whose Taylor scratch is resident at once (the segment is formed in chunks)
  int uplanes = 4;  // planes per propagator slot: U (2), or U and the gate tree's second half (4)
  int R = 1, Q = 1;
  int chunk = 0;  // slices per gradient chunk
  int nslots = 0;
  size_t elem = 8;
  // workspace layout (bytes)
  size_t off_flags = 0, off_ent = 0, off_T = 0, off_gacc = 0, off_sync = 0, off_xchg = 0, bytes = 0;
  long long xchg_words = 0;  // per direction
  bool coop = false;      // co-operative sweeps (several work-groups per job)
  bool coop_serial = false;  // ... whose two directions do not fit on the CUs together
  int coop_w = 1;         // largest number of work-groups of a job
  size_t coop_lds = 0;    // dynamic LDS of the co-operative sweep (bytes)
  long long expm_items = 0, panel_items = 0;
  long long entries_per_seg = 0;
  int max_mp = 0;         // largest padded block
  bool small_grad = false;  // every block <= 64 wide: the one-wave gradient series
  size_t sweep_lds_elems = 0;
  int max_cc = 0;
  long long total_u = 0, total_D = 0, total_U = 0;
  std::vector<qoc::JobDev> jobs;
  std::vector<qoc::ProbDev> probs;
  std::vector<qoc::PanelDesc> panels;
  qoc::DeviceBuffer d_jobs, d_probs, d_panels;
  qoc::DeviceBuffer d_theta, d_w;
  int grid_gemm = 512;
  int variant = 0;        // GEMM tile variant (index into the precision's table)
  int sweep_mode = 0;     // QOC_SWEEP_* bits (qoc_plan_set_sweep_mode)
  int gen_split = 0;      // generator column ranges (0: automatic; qoc_plan_set_generator_split)
  int ncu = 256;
  hipStream_t st2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // A batched plan whose propagators do not all fit the budget at once is run as groups of
  // consecutive problems, each a plan of its own whose propagators fit (no recompute), one
  // after another in the same workspace; a problem too large on its own is a group that
  // segments.  This plan's own tables still describe every job (slice statistics, sizes).
  std::vector<qoc_plan_s*> groups;
  std::vector<int> grp_prob0;  // first problem of each group
  ~qoc_plan_s() {
    for (auto* g : groups) delete g;
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (st2) (void)hipStreamDestroy(st2);
  }
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

// Evaluation scheme of a slice with ||X||_1 = nx: Paterson-Stockmeyer Taylor of degree
// q r (powers Y^2..Y^r, q-1 Horner products: r-1+q-1 products) or, q = 0, the four-product
// degree-12 scheme (A^2, A^3 and two products); then s squarings.  The cheapest in
// products wins; among Paterson-Stockmeyer degrees ties go to the larger one, and the
// degree-12 scheme wins a tie with them (the higher degree, and every such slice shares the
// same two launches).  The degree-12 scheme is offered only when t12 is set (FP32 plans:
// its epilogues move more data per product, which the FP64 accumulator layout makes four
// times as costly, and its products of non-unitary intermediates raise the unitarity error
// about threefold).  pow_free products (Y^2, Y^3) come from the generator and cost nothing
// here.
__host__ __device__ inline void pick_degree(double nx, const double* theta, int r, int qmax, int t12, int pow_free,
                                            int* q_out, int* s_out) {
  int best_q = qmax, best_s = 0, best_cost = 1 << 30;
  for (int q = qmax; q >= 1; --q) {
    int sq = 0;
    while (sq < 62 && nx > ldexp(theta[q * r], sq)) ++sq;
    const int cost = (r - 1 - pow_free) + (q - 1) + sq;
    if (cost < best_cost) { best_cost = cost; best_q = q; best_s = sq; }
  }
  if (t12) {
    int s12 = 0;
    while (s12 < 62 && nx > ldexp(theta[12], s12)) ++s12;
    if (4 - pow_free + s12 <= best_cost) { best_q = 0; best_s = s12; }
  }
  *q_out = best_q;
  *s_out = best_s;
}

// The Horner chain of a degree-12 (q = 0) entry ends where a q = 1 chain would: in the
// first ping-pong buffer.
__host__ __device__ inline int qeff(int q) { return q > 0 ? q : 1; }

__constant__ double kInvFact[64];
__constant__ double kT12c[4][4];  // the degree-12 scheme's coefficients (taylor12.h)

// ===================================================================== generator + norm
// One work-group per job and group of GEN_SG slices.  Pass 1: FP64 column sums of
// |H_j| for every slice of the group (one wave per column, lanes over rows, each operator
// element read once for all slices), giving the exact 1-norms and each slice's (q, s).
// Pass 2: Y = -i dt 2^-s H_j in the working precision, again reading H once per group.
constexpr int GEN_SG = 8;
constexpr int kMaxPair = 15, kMaxTrip = 35;  // pair_count / triple_count at kMaxPowK

// Coefficients of the operator products for the group's slices, scale sc = dt 2^-s
// folded in: pair (a <= b) -sc^2 u_a u_b, triple (a <= b <= c) sc^3 u_a u_b u_c (u_0 = 1),
// lexicographic order as the products; in the working precision (the combinations of the
// products are formed in it, like the products they replace).
template <typename T>
__device__ inline void gen_product_coefs(int K, int ns, const double (*us)[kMaxControls + 1], const double* scale,
                                         T (*cp)[kMaxPair], T (*ct)[kMaxTrip]) {
  const int O = K + 1;
  for (int t = threadIdx.x; t < GEN_SG; t += blockDim.x) {
    const double sc = t < ns ? scale[t] : 0.0, sc2 = sc * sc, sc3 = sc2 * sc;
    int i = 0, j = 0;
    for (int a = 0; a < O; ++a)
      for (int b = a; b < O; ++b) cp[t][i++] = (T)(-sc2 * us[t][a] * us[t][b]);
    for (int a = 0; a < O; ++a)
      for (int b = a; b < O; ++b)
        for (int c = b; c < O; ++c) ct[t][j++] = (T)(sc3 * us[t][a] * us[t][b] * us[t][c]);
  }
}

// Pass 2 of the generator for one element idx of a job's block and the group's ns slices
// (chunk slots Y0 + t * ent_stride): Y = -i sc H_j with sc = dt 2^-s in slot 0; with the
// operator products (pw != null) also Y^2 = -sc^2 sum_ab u_a u_b S_ab in slot 1 and
// Y^3 = i sc^3 sum_abc u_a u_b u_c T_abc in slot 2.  When gen_init (FP32 plans, r = 3) the
// slice's first Taylor combinations are formed here too: for the degree-12 scheme (q = 0)
// B_i = sum_k c[i][k] Y^k (Y^0 = I) go to slots 0, 1, 2 (B1, B2, B3, in place of the powers,
// which that scheme needs no more) and r (B4); for Paterson-Stockmeyer (r = 3) the start
// T0 = c_{qr} Y^r + sum_{i<r} c_{(q-1)r+i} Y^i goes to slot r, or, for q = 1 and no
// squaring, T0 = U itself to the propagator storage.  FP64 arithmetic for Y,
// the working precision for the product combinations (like the products they replace).
template <typename T>
__device__ inline void gen_element(const JobDev& jb, size_t idx, int ns, int r, int gen_init, const T* pw,
                                   const double (*us)[kMaxControls + 1], const T (*cp)[kMaxPair],
                                   const T (*ct)[kMaxTrip], const double* scale, const int* qsl, const int* ssl,
                                   T* Y0, size_t ent_stride, T* U0) {
  const int m = jb.m, mp = jb.mp, K = jb.K;
  const size_t plane = (size_t)mp * mp;
  const double* H = jb.h64;
  const int rr = (int)(idx % mp), c = (int)(idx / mp);
  const bool in = rr < m && c < m;
  double hr[GEN_SG], hi[GEN_SG];
#pragma unroll
  for (int t = 0; t < GEN_SG; ++t) hr[t] = hi[t] = 0.0;
  if (in) {
    for (int o = 0; o <= K; ++o) {
      const double ar = ld_global<double>(H + (size_t)(2 * o) * plane + idx);
      const double ai = ld_global<double>(H + (size_t)(2 * o + 1) * plane + idx);
#pragma unroll
      for (int t = 0; t < GEN_SG; ++t) {
        hr[t] += us[t][o] * ar;
        hi[t] += us[t][o] * ai;
      }
    }
  }
  if (!pw) {
    // -i * scale * (hr + i hi) = scale * hi - i scale * hr
#pragma unroll
    for (int t = 0; t < GEN_SG; ++t) {
      if (t < ns) {
        T* Y = Y0 + (size_t)t * ent_stride;
        Y[idx] = (T)(scale[t] * hi[t]);
        Y[idx + plane] = (T)(-scale[t] * hr[t]);
      }
    }
    return;
  }
  // Y^2 = sum cp S (cp carries -sc^2), Y^3 = i sum ct T (ct carries sc^3)
  T sr[GEN_SG], si[GEN_SG], cr[GEN_SG], ci[GEN_SG];
#pragma unroll
  for (int t = 0; t < GEN_SG; ++t) sr[t] = si[t] = cr[t] = ci[t] = T(0);
  if (in) {
    const int np = pair_count(K), nt = triple_count(K);
#pragma unroll 2
    for (int i = 0; i < np; ++i) {
      const T ar = ld_global<T>(pw + (size_t)(2 * i) * plane + idx);
      const T ai = ld_global<T>(pw + (size_t)(2 * i + 1) * plane + idx);
#pragma unroll
      for (int t = 0; t < GEN_SG; ++t) {
        sr[t] += cp[t][i] * ar;
        si[t] += cp[t][i] * ai;
      }
    }
#pragma unroll 2
    for (int i = 0; i < nt; ++i) {
      const size_t o = (size_t)(2 * (np + i)) * plane + idx;
      const T ar = ld_global<T>(pw + o), ai = ld_global<T>(pw + o + plane);
#pragma unroll
      for (int t = 0; t < GEN_SG; ++t) {
        cr[t] += ct[t][i] * ar;
        ci[t] += ct[t][i] * ai;
      }
    }
  }
  const bool diag = rr == c && rr < m;
#pragma unroll
  for (int t = 0; t < GEN_SG; ++t) {
    if (t >= ns) continue;
    const double sc = scale[t];
    const double y1r = sc * hi[t], y1i = -sc * hr[t];
    const double y2r = sr[t], y2i = si[t];
    const double y3r = -(double)ci[t], y3i = cr[t];
    T* Y = Y0 + (size_t)t * ent_stride;
    const int q = gen_init ? qsl[t] : 1;
    if (gen_init && q == 0) {
      // degree-12 scheme: B1, B2, B3 into slots 0..2, B4 into slot r
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const double vr = kT12c[b][1] * y1r + kT12c[b][2] * y2r + kT12c[b][3] * y3r + (diag ? kT12c[b][0] : 0.0);
        const double vi = kT12c[b][1] * y1i + kT12c[b][2] * y2i + kT12c[b][3] * y3i;
        const size_t sl = b < 3 ? (size_t)b : (size_t)r;
        Y[(2 * sl) * plane + idx] = (T)vr;
        Y[(2 * sl + 1) * plane + idx] = (T)vi;
      }
      continue;
    }
    Y[idx] = (T)y1r;
    Y[plane + idx] = (T)y1i;
    Y[2 * plane + idx] = (T)y2r;
    Y[3 * plane + idx] = (T)y2i;
    Y[4 * plane + idx] = (T)y3r;
    Y[5 * plane + idx] = (T)y3i;
    if (!gen_init) continue;
    const double c0 = kInvFact[(q - 1) * 3], c1 = kInvFact[(q - 1) * 3 + 1], c2 = kInvFact[(q - 1) * 3 + 2],
                 c3 = kInvFact[q * 3];
    const double vr = c1 * y1r + c2 * y2r + c3 * y3r + (diag ? c0 : 0.0);
    const double vi = c1 * y1i + c2 * y2i + c3 * y3i;
    if (q == 1 && ssl[t] == 0) {
      // degree 3, no squaring: T0 is the propagator
      T* U = U0 + (size_t)t * jb.uslot;
      U[idx] = (T)vr;
      U[idx + plane] = (T)vi;
    } else {
      Y[(size_t)(2 * r) * plane + idx] = (T)vr;
      Y[(size_t)(2 * r + 1) * plane + idx] = (T)vi;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_generator(const JobDev* jobs, int njobs, const double* u, int seg_j0,
                                                   int seg_len, int c0, int clen, int groups, char* ws, size_t off_T,
                                                   int* ent_s,
                                                   int* ent_q, double* ent_norm, int* flags, const double* theta,
                                                   int r, int qmax, int t12, int pow_free, int smax, double norm_bound,
                                                   int skip_n) {
  __shared__ double red[GEN_SG][256];
  __shared__ double us[GEN_SG][kMaxControls + 1];
  __shared__ T cp[GEN_SG][kMaxPair], ct[GEN_SG][kMaxTrip];
  __shared__ double scale[GEN_SG];
  __shared__ int qsl[GEN_SG], ssl[GEN_SG];
  const int J = blockIdx.x / groups, g = blockIdx.x % groups;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  if (jb.N <= skip_n) return;  // recompute pass: this job's propagators are still resident
  const int jl0 = c0 + g * GEN_SG;  // slices jl0 .. of the segment; chunk slots jl0 - c0 ..
  const int len = min(job_len(jb, seg_j0, seg_len), c0 + clen);
  if (jl0 >= len) return;
  const int ns = min(GEN_SG, len - jl0);
  const int m = jb.m, mp = jb.mp, K = jb.K;
  const size_t plane = (size_t)mp * mp;
  const double* H = jb.h64;
  const double* uj = u + jb.u_off;
  for (int idx = threadIdx.x; idx < GEN_SG * (K + 1); idx += blockDim.x) {
    const int t = idx / (K + 1), o = idx % (K + 1);
    double v = 0.0;
    if (t < ns) v = o == 0 ? 1.0 : uj[(size_t)(seg_j0 + jl0 + t) * K + (o - 1)];
    us[t][o] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double cmax[GEN_SG];
#pragma unroll
  for (int t = 0; t < GEN_SG; ++t) cmax[t] = 0.0;
  for (int c = wave; c < m; c += nw) {
    double cs[GEN_SG];
#pragma unroll
    for (int t = 0; t < GEN_SG; ++t) cs[t] = 0.0;
    for (int rr = lane; rr < m; rr += 64) {
      const size_t idx = (size_t)rr + (size_t)c * mp;
      double hr[GEN_SG], hi[GEN_SG];
#pragma unroll
      for (int t = 0; t < GEN_SG; ++t) hr[t] = hi[t] = 0.0;
      for (int o = 0; o <= K; ++o) {
        const double ar = ld_global<double>(H + (size_t)(2 * o) * plane + idx);
        const double ai = ld_global<double>(H + (size_t)(2 * o + 1) * plane + idx);
#pragma unroll
        for (int t = 0; t < GEN_SG; ++t) {
          hr[t] += us[t][o] * ar;
          hi[t] += us[t][o] * ai;
        }
      }
#pragma unroll
      for (int t = 0; t < GEN_SG; ++t) cs[t] += hypot(hr[t], hi[t]);
    }
#pragma unroll
    for (int t = 0; t < GEN_SG; ++t) cmax[t] = fmax(cmax[t], warp_sum(cs[t]));
  }
#pragma unroll
  for (int t = 0; t < GEN_SG; ++t) red[t][threadIdx.x] = cmax[t];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int t = 0; t < GEN_SG; ++t) red[t][threadIdx.x] = fmax(red[t][threadIdx.x], red[t][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < ns) {
    const int t = threadIdx.x;
    const long long e = jb.ent_off + jl0 + t;
    const double nx = jb.dt * red[t][0];
    bool finite = isfinite(nx);
    for (int o = 1; o <= K; ++o) finite = finite && isfinite(us[t][o]);
    int flag = 0;
    if (!finite) flag |= 2;
    if (nx > norm_bound * (1.0 + 1e-12)) flag |= 1;
    int best_q, best_s;
    pick_degree(nx, theta, r, qmax, t12, pow_free, &best_q, &best_s);
    if (best_s > smax) { flag |= 1; best_s = smax; }
    if (flag) atomicOr(flags, flag);
    atomicMax(flags + 1, best_s);
    atomicMax(flags + 2, best_q);
    ent_s[e] = best_s;
    ent_q[e] = best_q;
    ent_norm[e] = nx;
    scale[t] = ldexp(jb.dt, -best_s);
    qsl[t] = best_q;
    ssl[t] = best_s;
  }
  __syncthreads();
  const T* pw = pow_free ? job_products<T>(jb, ws, off_T) : nullptr;
  if (pw) gen_product_coefs<T>(K, ns, us, scale, cp, ct);
  __syncthreads();
  const size_t ent_stride = (size_t)(r + 2) * 2 * plane;
  T* Y0 = tplane<T>(ws, off_T, jb.sbuf_off) + (size_t)(jl0 - c0) * ent_stride;
  T* U0 = tplane<T>(ws, off_T, jb.ubuf_off) + (size_t)jl0 * jb.uslot;
  const int gen_init = pow_free && r == 3;
  for (size_t idx = threadIdx.x; idx < plane; idx += blockDim.x)
    gen_element<T>(jb, idx, ns, r, gen_init, pw, us, cp, ct, scale, qsl, ssl, Y0, ent_stride, U0);
}

// The same generator split over column ranges, for chunks with too few (job, slice group)
// pairs to fill the GPU (short pulses on large blocks): k_gen_norms takes the largest
// column sum of |H_j| over csplit column ranges (atomic maximum on the bit pattern of a
// non-negative double, ent_norm zeroed first), k_gen_pick turns it into each slice's
// (q, s) and flags, k_gen_form writes Y over csplit element ranges.  Same arithmetic as
// k_generator, element by element.
__device__ inline void gen_load_controls(const JobDev& jb, const double* u, int seg_j0, int jl0, int ns,
                                         double (*us)[kMaxControls + 1]) {
  const int K = jb.K;
  const double* uj = u + jb.u_off;
  for (int idx = threadIdx.x; idx < GEN_SG * (K + 1); idx += blockDim.x) {
    const int t = idx / (K + 1), o = idx % (K + 1);
    double v = 0.0;
    if (t < ns) v = o == 0 ? 1.0 : uj[(size_t)(seg_j0 + jl0 + t) * K + (o - 1)];
    us[t][o] = v;
  }
}

// zero the chunk's entries c0 .. c0 + clen - 1 of every job (the maxima of k_gen_norms)
__global__ void k_gen_zero(const JobDev* jobs, int njobs, int c0, int clen, double* ent_norm) {
  for (int J = blockIdx.y; J < njobs; J += gridDim.y)
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < clen; t += gridDim.x * blockDim.x)
      ent_norm[jobs[J].ent_off + c0 + t] = 0.0;
}

__global__ void __launch_bounds__(256) k_gen_norms(const JobDev* jobs, int njobs, const double* u, int seg_j0,
                                                   int seg_len, int c0, int clen, int groups, int csplit,
                                                   double* ent_norm, int skip_n) {
  __shared__ double red[GEN_SG][256];
  __shared__ double us[GEN_SG][kMaxControls + 1];
  const int J = blockIdx.x / (groups * csplit), g = (blockIdx.x / csplit) % groups, cs = blockIdx.x % csplit;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  if (jb.N <= skip_n) return;
  const int jl0 = c0 + g * GEN_SG;
  const int len = min(job_len(jb, seg_j0, seg_len), c0 + clen);
  if (jl0 >= len) return;
  const int ns = min(GEN_SG, len - jl0);
  const int m = jb.m, mp = jb.mp, K = jb.K;
  const int cw = (m + csplit - 1) / csplit, clo = cs * cw, chi = min(m, clo + cw);
  const size_t plane = (size_t)mp * mp;
  const double* H = jb.h64;
  gen_load_controls(jb, u, seg_j0, jl0, ns, us);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double cmax[GEN_SG];
#pragma unroll
  for (int t = 0; t < GEN_SG; ++t) cmax[t] = 0.0;
  for (int c = clo + wave; c < chi; c += nw) {
    double cs_[GEN_SG];
#pragma unroll
    for (int t = 0; t < GEN_SG; ++t) cs_[t] = 0.0;
    for (int rr = lane; rr < m; rr += 64) {
      const size_t idx = (size_t)rr + (size_t)c * mp;
      double hr[GEN_SG], hi[GEN_SG];
#pragma unroll
      for (int t = 0; t < GEN_SG; ++t) hr[t] = hi[t] = 0.0;
      for (int o = 0; o <= K; ++o) {
        const double ar = ld_global<double>(H + (size_t)(2 * o) * plane + idx);
        const double ai = ld_global<double>(H + (size_t)(2 * o + 1) * plane + idx);
#pragma unroll
        for (int t = 0; t < GEN_SG; ++t) {
          hr[t] += us[t][o] * ar;
          hi[t] += us[t][o] * ai;
        }
      }
#pragma unroll
      for (int t = 0; t < GEN_SG; ++t) cs_[t] += hypot(hr[t], hi[t]);
    }
#pragma unroll
    for (int t = 0; t < GEN_SG; ++t) cmax[t] = fmax(cmax[t], warp_sum(cs_[t]));
  }
#pragma unroll
  for (int t = 0; t < GEN_SG; ++t) red[t][threadIdx.x] = cmax[t];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int t = 0; t < GEN_SG; ++t) red[t][threadIdx.x] = fmax(red[t][threadIdx.x], red[t][threadIdx.x + w]);
    __syncthreads();
  }
  if ((int)threadIdx.x < ns)
    atomicMax(reinterpret_cast<unsigned long long*>(ent_norm + jb.ent_off + jl0 + threadIdx.x),
              (unsigned long long)__double_as_longlong(red[threadIdx.x][0]));
}

__global__ void k_gen_pick(const JobDev* jobs, int njobs, const double* u, int seg_j0, int seg_len, int c0, int clen,
                           int groups, int* ent_s, int* ent_q, double* ent_norm, int* flags, const double* theta, int r,
                           int qmax, int t12, int pow_free, int smax, double norm_bound, int skip_n) {
  const int J = blockIdx.x / groups, g = blockIdx.x % groups;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  if (jb.N <= skip_n) return;
  const int jl0 = c0 + g * GEN_SG;
  const int len = min(job_len(jb, seg_j0, seg_len), c0 + clen);
  const int t = threadIdx.x;
  if (t >= GEN_SG || jl0 + t >= len) return;
  const long long e = jb.ent_off + jl0 + t;
  const double nx = jb.dt * ent_norm[e];
  bool finite = isfinite(nx);
  for (int o = 0; o < jb.K; ++o) finite = finite && isfinite(u[jb.u_off + (size_t)(seg_j0 + jl0 + t) * jb.K + o]);
  int flag = 0;
  if (!finite) flag |= 2;
  if (nx > norm_bound * (1.0 + 1e-12)) flag |= 1;
  int best_q, best_s;
  pick_degree(nx, theta, r, qmax, t12, pow_free, &best_q, &best_s);
  if (best_s > smax) { flag |= 1; best_s = smax; }
  if (flag) atomicOr(flags, flag);
  atomicMax(flags + 1, best_s);
  atomicMax(flags + 2, best_q);
  ent_s[e] = best_s;
  ent_q[e] = best_q;
  ent_norm[e] = nx;
}

template <typename T>
__global__ void __launch_bounds__(256) k_gen_form(const JobDev* jobs, int njobs, const double* u, int seg_j0,
                                                  int seg_len, int c0, int clen, int groups, int csplit, char* ws,
                                                  size_t off_T, const int* ent_s, const int* ent_q, int r,
                                                  int pow_free, int skip_n) {
  __shared__ double us[GEN_SG][kMaxControls + 1];
  __shared__ T cp[GEN_SG][kMaxPair], ct[GEN_SG][kMaxTrip];
  __shared__ double scale[GEN_SG];
  __shared__ int qsl[GEN_SG], ssl[GEN_SG];
  const int J = blockIdx.x / (groups * csplit), g = (blockIdx.x / csplit) % groups, cs = blockIdx.x % csplit;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  if (jb.N <= skip_n) return;
  const int jl0 = c0 + g * GEN_SG;
  const int len = min(job_len(jb, seg_j0, seg_len), c0 + clen);
  if (jl0 >= len) return;
  const int ns = min(GEN_SG, len - jl0);
  const int mp = jb.mp, K = jb.K;
  const size_t plane = (size_t)mp * mp;
  const size_t ew = (plane + csplit - 1) / csplit, lo = cs * ew, hi_ = min(plane, lo + ew);
  gen_load_controls(jb, u, seg_j0, jl0, ns, us);
  if ((int)threadIdx.x < ns) {
    const long long e = jb.ent_off + jl0 + threadIdx.x;
    scale[threadIdx.x] = ldexp(jb.dt, -ent_s[e]);
    qsl[threadIdx.x] = ent_q[e];
    ssl[threadIdx.x] = ent_s[e];
  }
  __syncthreads();
  const T* pw = pow_free ? job_products<T>(jb, ws, off_T) : nullptr;
  if (pw) gen_product_coefs<T>(K, ns, us, scale, cp, ct);
  __syncthreads();
  const size_t ent_stride = (size_t)(r + 2) * 2 * plane;
  T* Y0 = tplane<T>(ws, off_T, jb.sbuf_off) + (size_t)(jl0 - c0) * ent_stride;
  T* U0 = tplane<T>(ws, off_T, jb.ubuf_off) + (size_t)jl0 * jb.uslot;
  const int gen_init = pow_free && r == 3;
  for (size_t idx = lo + threadIdx.x; idx < hi_; idx += blockDim.x)
    gen_element<T>(jb, idx, ns, r, gen_init, pw, us, cp, ct, scale, qsl, ssl, Y0, ent_stride, U0);
}

// ===================================================================== expm GEMM steps
enum { STEP_POWER = 0, STEP_HORNER = 1, STEP_SQUARE = 2, STEP_T12 = 3 };

// One product step over every entry of a chunk of the segment (persistent, XCD-grouped
// items).  Taylor scratch of an entry (one slot per chunk slice): 0 = Y, i-1 = Y^i (i <= r),
// r and r+1 = ping-pong T.  The last power step also forms the Horner start T0; the last
// product of an entry writes U into the segment's propagator storage.
// One tile product of the propagator formation: operands, where the result goes.
template <typename T>
struct ExpmItem {
  TileOperands<T> op;
  T* base;   // Taylor scratch of the entry's chunk slot
  T* ubase;  // U of the entry
  int m, ic, se, qe;
};

template <typename Shape>
__global__ void __launch_bounds__(256, Shape::WAVES)
    k_expm_step(const JobDev* jobs, int njobs, long long total_items, char* ws, size_t off_T, const int* ent_s,
                const int* ent_q, int mode, int step, int r, int seg_j0, int seg_len, int c0, int clen,
                int skip_n, const int* flags, int gen_b) {
  typedef typename Shape::T T;
  __shared__ TileSmem<Shape> lds;
  // a Horner or squaring step no entry needs (flags[2] is the largest q, flags[1] the
  // largest s the generator picked so far) exits at once instead of walking every item
  if ((mode == STEP_HORNER && step > flags[2] - 1) || (mode == STEP_SQUARE && step > flags[1])) return;
  const ItemRange rg = xcd_items(total_items);
  ItemCursor cur;
  // item -> tile product; false when this step has nothing to do for the item
  auto prep = [&](long long it, ExpmItem<T>& x) -> bool {
    const int J = cursor_find(jobs, njobs, it, cur);
    const JobDev jb = jobs[J];
    const long long local = it - jb.item_off;
    const int t2 = jb.tiles_m * jb.tiles_n;
    const int jc = (int)(local / t2);  // slot in the chunk
    const int jl = c0 + jc;            // slice of the segment
    if (jc >= clen || jl >= job_len(jb, seg_j0, seg_len) || jb.N <= skip_n) return false;
    const int tile = (int)(local % t2);
    const int ti = tile / jb.tiles_n, tj = tile % jb.tiles_n;
    const long long e = jb.ent_off + jl;
    const int se = ent_s[e], qe = ent_q[e];
    const bool t12 = qe == 0;  // the four-product degree-12 scheme
    int ia, ib, ic;
    if (mode == STEP_POWER) {
      if (t12 && step > 3) return false;  // it needs Y^2 and Y^3 only
      ia = step - 2; ib = 0; ic = step - 1;
      // Y is skew-Hermitian, so Y^step is Hermitian or skew-Hermitian: tiles wholly above
      // the diagonal are written as mirrors by the tiles below it (except when this step
      // also forms the entry's final propagator, which has no such symmetry)
      const bool fin = !t12 && step == r && qe == 1 && se == 0;
      if (!fin && ti * Shape::BM + Shape::BM <= tj * Shape::BN) return false;
    } else if (mode == STEP_T12) {
      if (!t12) return false;
      if (step == 1) {  // B4 B4 (B4 in buffer r) -> A6 = B3 + B4^2 in buffer r+1
        ia = r; ib = r; ic = r + 1;
      } else {          // (B2 + A6) A6 + B1 -> T12 in buffer r
        ia = 1; ib = r + 1; ic = r;
      }
    } else if (mode == STEP_HORNER) {
      if (qe - 1 < step) return false;
      ia = r + ((step - 1) & 1); ib = r - 1; ic = r + (step & 1);
    } else {
      if (se < step) return false;
      const int h = qeff(qe) - 1 + step - 1;
      ia = r + (h & 1); ib = ia; ic = r + ((h + 1) & 1);
    }
    const int mp = jb.mp;
    const size_t plane = (size_t)mp * mp;
    x.base = tplane<T>(ws, off_T, jb.sbuf_off) + (size_t)jc * (size_t)(r + 2) * 2 * plane;
    x.ubase = tplane<T>(ws, off_T, jb.ubuf_off) + (size_t)jl * jb.uslot;
    x.m = jb.m;
    x.ic = ic;
    x.se = se;
    x.qe = qe;
    x.op.A = x.base + (size_t)ia * 2 * plane;
    x.op.a_ps = plane;
    x.op.lda = mp;
    x.op.B = x.base + (size_t)ib * 2 * plane;
    x.op.b_ps = plane;
    x.op.ldb = mp;
    x.op.M = mp;
    x.op.N = mp;
    x.op.K = mp;
    x.op.row0 = ti * Shape::BM;
    x.op.col0 = tj * Shape::BN;
    return true;
  };
  long long it = rg.begin;
  ExpmItem<T> x;
  while (it < rg.end && !prep(it, x)) it += rg.step;
  if (it >= rg.end) return;
  TilePipe pipe = tile_start<Shape>(x.op, lds);
  for (;;) {
    long long nx = it + rg.step;
    ExpmItem<T> xn = x;
    while (nx < rg.end && !prep(nx, xn)) nx += rg.step;
    const bool more = nx < rg.end;
    TileAcc<Shape> acc;
    tile_mma<Shape>(x.op, lds, acc, pipe, more, xn.op);
    const int se = x.se, qe = x.qe, ic = x.ic;
    const bool t12 = qe == 0;
    const bool final_op = (mode == STEP_SQUARE && step == se) || (mode == STEP_HORNER && se == 0 && step == qe - 1) ||
                          (mode == STEP_T12 && step == 2 && se == 0);
    const int mp = x.op.M;
    const size_t plane = (size_t)mp * mp;
    T* const base = x.base;
    T* const ubase = x.ubase;
    T* C = final_op ? ubase : base + (size_t)ic * 2 * plane;  // the last product of an entry is U
    double coef[8];
    double ctop = 0.0;
    const int lh = qe - 1 - step;
    const bool init_T = mode == STEP_POWER && step == r && !t12;
    const bool init_final = init_T && qe == 1 && se == 0;
    const bool init_B4 = mode == STEP_POWER && step == 3 && t12;
    // power steps (but a final one) keep the elements on and below the diagonal and write
    // the mirror images of those strictly below; Y^step has the symmetry sign psign
    // (M[c][r] = psign conj(M[r][c]))
    const bool sym = mode == STEP_POWER && !init_final;
    const T psign = (step & 1) ? T(-1) : T(1);
    if (mode == STEP_HORNER)
      for (int i = 0; i < r; ++i) coef[i] = kInvFact[lh * r + i];
    if (init_T) {
      ctop = kInvFact[qe * r];
      for (int i = 0; i < r; ++i) coef[i] = kInvFact[(qe - 1) * r + i];
    }
    typedef typename Vec4<T>::type V4;
#pragma unroll
    for (int ri = 0; ri < Shape::SM; ++ri)
#pragma unroll
      for (int ci = 0; ci < Shape::SN; ++ci) {
        const int rbase = acc_row_base<Shape>(x.op.row0, ri);
        const int col = acc_col<Shape>(x.op.col0, ci);
        if (rbase >= mp || col >= mp) continue;
        const int row0 = rbase + acc_row_off<T>(0);  // this lane's first accumulator row
        const size_t at = (size_t)row0 + (size_t)col * mp;
        const int cb = col - (int)(threadIdx.x & 15);  // first column of the sub-tile
        if (sym && rbase + 16 <= cb) continue;        // above the diagonal: mirrored from below
        const bool below = rbase >= cb + 16;           // every element strictly below
        // direct store of the elements on or below the diagonal of a symmetric step, plus the
        // conjugates of (mr, mi) at the transposed positions of those strictly below
        auto put = [&](T* P, const V4& wr, const V4& wi, const V4& mr, const V4& mi) {
          if (!sym || below) {
            acc_store<T>(P + at, wr);
            acc_store<T>(P + at + plane, wi);
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (row0 + v * AccRowStep<T>::value >= col) {
                P[at + v * AccRowStep<T>::value] = wr[v];
                P[at + plane + v * AccRowStep<T>::value] = wi[v];
              }
          }
          if (!sym) return;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int rr = row0 + v * AccRowStep<T>::value;
            if (below || rr > col) {
              T* d = P + (size_t)col + (size_t)rr * mp;
              d[0] = mr[v];
              d[plane] = -mi[v];
            }
          }
        };
        V4 vr = acc.re[ri][ci], vi = acc.im[ri][ci];
        if (mode == STEP_HORNER) {
          for (int i = 1; i < r; ++i) {
            const T* Pp = base + (size_t)(i - 1) * 2 * plane + at;
            vr += (T)coef[i] * acc_load<T>(Pp);
            vi += (T)coef[i] * acc_load<T>(Pp + plane);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (row0 + v * AccRowStep<T>::value == col && col < x.m) vr[v] += (T)coef[0];
        }
        if (mode == STEP_T12 && gen_b) {
          // the generator wrote B1, B2, B3 into buffers 0..2
          if (step == 1) {
            // A6 = B3 + B4^2 (the product); buffer 1 <- B2 + A6 (not an operand of this step)
            vr += acc_load<T>(base + 4 * plane + at);
            vi += acc_load<T>(base + 5 * plane + at);
            acc_store<T>(base + 2 * plane + at, acc_load<T>(base + 2 * plane + at) + vr);
            acc_store<T>(base + 3 * plane + at, acc_load<T>(base + 3 * plane + at) + vi);
          } else {
            // T12 = B1 (buffer 0) + (B2 + A6) A6
            vr += acc_load<T>(base + at);
            vi += acc_load<T>(base + at + plane);
          }
        } else if (mode == STEP_T12) {
          // sum_k c[k] P_k at this tile for P_0 = I, P_1..3 = Y, Y^2, Y^3 (buffers 0..2)
          const V4 y1r = acc_load<T>(base + at), y1i = acc_load<T>(base + at + plane);
          const V4 y2r = acc_load<T>(base + 2 * plane + at), y2i = acc_load<T>(base + 3 * plane + at);
          auto combo = [&](int i, V4& cr, V4& ci) {
            cr = (T)kT12c[i][1] * y1r;
            ci = (T)kT12c[i][1] * y1i;
            cr += (T)kT12c[i][2] * y2r;
            ci += (T)kT12c[i][2] * y2i;
            if (step == 1) {
              const V4 y3r = acc_load<T>(base + 4 * plane + at), y3i = acc_load<T>(base + 5 * plane + at);
              cr += (T)kT12c[i][3] * y3r;
              ci += (T)kT12c[i][3] * y3i;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (row0 + v * AccRowStep<T>::value == col && col < x.m) cr[v] += (T)kT12c[i][0];
          };
          if (step == 1) {
            // A6 = B3 + B4^2 (the product); buffer 0 <- B1, buffer 1 <- B2 + A6 (neither is an
            // operand of this step, and each tile rewrites only its own elements)
            V4 br, bi;
            combo(2, br, bi);
            vr += br;
            vi += bi;
            V4 b1r, b1i, b2r, b2i;
            combo(0, b1r, b1i);
            combo(1, b2r, b2i);
            acc_store<T>(base + at, b1r);
            acc_store<T>(base + at + plane, b1i);
            acc_store<T>(base + 2 * plane + at, b2r + vr);
            acc_store<T>(base + 3 * plane + at, b2i + vi);
          } else {
            // T12 = B1 (buffer 0) + (B2 + A6) A6
            vr += y1r;
            vi += y1i;
          }
        }
        put(C, vr, vi, psign * vr, psign * vi);
        if (init_B4) {
          // B4 = sum_k c[3][k] P_k (the product is Y^3) into buffer r: the degree-12 scheme's start
          const V4 y1r = acc_load<T>(base + at), y1i = acc_load<T>(base + at + plane);
          const V4 y2r = acc_load<T>(base + 2 * plane + at), y2i = acc_load<T>(base + 3 * plane + at);
          V4 br = (T)kT12c[3][3] * vr, bi = (T)kT12c[3][3] * vi;
          br += (T)kT12c[3][1] * y1r + (T)kT12c[3][2] * y2r;
          bi += (T)kT12c[3][1] * y1i + (T)kT12c[3][2] * y2i;
          // mirror: B4[c][r] = conj(-c1 Y + c2 Y^2 - c3 Y^3)[r][c] off the diagonal
          const V4 mr = (T)kT12c[3][2] * y2r - (T)kT12c[3][1] * y1r - (T)kT12c[3][3] * vr;
          const V4 mi = (T)kT12c[3][2] * y2i - (T)kT12c[3][1] * y1i - (T)kT12c[3][3] * vi;
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (row0 + v * AccRowStep<T>::value == col && col < x.m) br[v] += (T)kT12c[3][0];
          put(base + (size_t)r * 2 * plane, br, bi, mr, mi);
        }
        if (init_T) {
          // T0 = c_{qr} Y^r + sum_{i<r} c_{(q-1)r+i} Y^i at this tile (the Horner start); its
          // mirror T0[c][r] = conj(sum_i (-1)^i c_i Y^i)[r][c] off the diagonal
          V4 tr = (T)ctop * vr, ti = (T)ctop * vi;
          V4 mr = psign * tr, mi = psign * ti;
          for (int i = 1; i < r; ++i) {
            const T* Pp = base + (size_t)(i - 1) * 2 * plane + at;
            const V4 pr = acc_load<T>(Pp), pi = acc_load<T>(Pp + plane);
            const T ci = (T)coef[i], cm = (i & 1) ? -ci : ci;
            tr += ci * pr;
            ti += ci * pi;
            mr += cm * pr;
            mi += cm * pi;
          }
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (row0 + v * AccRowStep<T>::value == col && col < x.m) tr[v] += (T)coef[0];
          put(init_final ? ubase : base + (size_t)r * 2 * plane, tr, ti, mr, mi);
        }
      }
    if (!more) break;
    it = nx;
    x = xn;
  }
}

// U of slice jl of the segment (the sweeps read U itself in both directions)
template <typename T>
__device__ inline const T* entry_U(const JobDev& jb, char* ws, size_t off_T, int jl) {
  return tplane<T>(ws, off_T, jb.ubuf_off) + (size_t)jl * jb.uslot;
}

// ===================================================================== state set-up
// psi0 -> forward store column 0, psi_f -> costate column N-1 (planar, working precision)
template <typename T>
__global__ void k_states_in(const JobDev* jobs, int njobs, const double2* psi0, const double2* psif, char* ws,
                            size_t off_T, int* flags) {
  for (int J = blockIdx.y; J < njobs; J += gridDim.y) {
  const JobDev jb = jobs[J];
  const int N = jb.N;
  const long long ncol_psi = (long long)(N + 1) * jb.d, ncol_lam = (long long)N * jb.d;
  T* Pp = tplane<T>(ws, off_T, jb.psi_off);
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
    const size_t cp = (size_t)c * jb.mp + i;
    const size_t cl = ((size_t)(N - 1) * jb.d + c) * jb.mp + i;
    Pp[cp] = (T)a.x;
    Pp[cp + pps] = (T)a.y;
    Lm[cl] = (T)b.x;
    Lm[cl + lps] = (T)b.y;
  }
  }
}

__global__ void k_zero_ints(int* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_fold_flags(const int* flags, int nprob, double* out) {
  for (int p = threadIdx.x; p < nprob; p += blockDim.x) {
    const int fl = (int)out[(size_t)p * 8 + 7] | flags[0];
    out[(size_t)p * 8 + 7] = (double)fl;
  }
}

// One state of problem p's sweeps as block panels (interleaved complex128): which = 0 the
// forward state psi_j (store column j, 0 <= j <= N), which = 1 the costate lambda_j (store
// column j - 1, 1 <= j <= N).
template <typename T>
__global__ void k_export_state(const JobDev* jobs, int job_begin, int job_end, const char* ws, size_t off_T,
                               int which, int j, double2* out) {
  for (int J = job_begin + blockIdx.y; J < job_end; J += gridDim.y) {
    const JobDev jb = jobs[J];
    const T* S = reinterpret_cast<const T*>(ws + off_T) + (which == 0 ? jb.psi_off : jb.lam_off);
    const size_t ncol = which == 0 ? (size_t)(jb.N + 1) * jb.d : (size_t)jb.N * jb.d;
    const size_t ps = (size_t)jb.mp * ncol;
    const size_t col = which == 0 ? (size_t)j : (size_t)(j - 1);
    const long long base = jb.state_off - jobs[job_begin].state_off;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < jb.m * jb.d; idx += gridDim.x * blockDim.x) {
      const int c = idx / jb.m, i = idx % jb.m;
      const size_t g = (col * jb.d + c) * jb.mp + i;
      out[base + (long long)c * jb.m + i] = make_double2((double)S[g], (double)S[g + ps]);
    }
  }
}

// ===================================================================== sweeps
// Sweep through one segment, one work-group (16 waves) per job, the state in LDS.
// DIR 0: psi_{j+1} = U_j psi_j, streaming U column by column: a lane owns 16 bytes of
// consecutive rows, a wave 64 such row vectors and one of G k-ranges; loads are unrolled
// so that many bytes are in flight per lane; partial sums meet in LDS.  DIR 1 (lambda_j =
// U_j^dag lambda_{j+1}) reads the same stored U as dot products down its columns
// (sweep_solo_bwd and the *_bwd variants below): only U is kept per slice.
template <typename T> struct SweepUnroll { static constexpr int value = 8; };
template <> struct SweepUnroll<double> { static constexpr int value = 4; };

// Sweep work split: a lane owns 16 bytes of consecutive rows (4 FP32 / 2 FP64), a wave a
// row group of 64 such; the 16 waves cover R row groups x G column (k) groups.
__host__ __device__ inline int sweep_rows_per_group(int elem) { return 64 * (16 / elem); }
__host__ __device__ inline int sweep_kgroups(int mp, int elem) {
  const int R = (mp + sweep_rows_per_group(elem) - 1) / sweep_rows_per_group(elem);
  return R >= 16 ? 1 : 16 / R;
}

// One work-group sweeps one job through the segment: 16 waves split the rows and the
// columns of U_j; the state and the partial sums live in LDS.
template <typename T, int DIR>
__device__ void sweep_solo(const JobDev& jb, char* ws, size_t off_T, const int* ent_s, const int* ent_q, int r,
                           int seg_j0, int seg_len) {
  static_assert(DIR == 0, "the backward one-group sweep is sweep_solo_bwd");
  typedef typename Vec16<T>::type TV;
  typedef typename Vec4<T>::type T4;
  constexpr int UNR = SweepUnroll<T>::value, RPL = Vec16<T>::n;
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  const int len = job_len(jb, seg_j0, seg_len);
  if (len <= 0) return;
  const int m = jb.m, mp = jb.mp, d = jb.d, N = jb.N;
  const int RG = sweep_rows_per_group((int)sizeof(T));
  const int R = (mp + RG - 1) / RG, G = sweep_kgroups(mp, (int)sizeof(T));
  T* sre = reinterpret_cast<T*>(smem_raw);  // state [d][mp]
  T* sim = sre + (size_t)d * mp;
  T* pre = sim + (size_t)d * mp;             // partial sums [G][d][mp]
  T* pim = pre + (size_t)G * d * mp;
  T* S = tplane<T>(ws, off_T, DIR == 0 ? jb.psi_off : jb.lam_off);
  const size_t ncol = DIR == 0 ? (size_t)(N + 1) * d : (size_t)N * d;
  const size_t ps = (size_t)mp * ncol;
  const int col_in = DIR == 0 ? seg_j0 : seg_j0 + len - 1;
  for (int idx = threadIdx.x; idx < mp * d; idx += blockDim.x) {
    const int c = idx / mp, i = idx % mp;
    const size_t g = ((size_t)col_in * d + c) * mp + i;
    sre[idx] = S[g];
    sim[idx] = S[g + ps];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kchunk = ((m + G - 1) / G + UNR - 1) / UNR * UNR;
  const size_t plane = (size_t)mp * mp;
  for (int it = 0; it < len; ++it) {
    const int jl = DIR == 0 ? it : len - 1 - it;
    const T* U = entry_U<T>(jb, ws, off_T, jl);
    for (int task = wave; task < R * G; task += 16) {
      const int rg = task % R, kg = task / R;
      const int i0 = rg * RG + RPL * lane;  // rows i0 .. i0 + RPL - 1 (mp is a multiple of 16)
      const int k0 = kg * kchunk, k1 = min(m, k0 + kchunk);
      T a[2][2][RPL];  // [copy][re, im][row]
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int t = 0; t < RPL; ++t) a[c][0][t] = a[c][1][t] = T(0);
      if (i0 < m) {
        const T* col = U + i0;
        int k = k0;
        for (; k + UNR <= k1; k += UNR) {
          TV ur[UNR], ui[UNR];
#pragma unroll
          for (int q = 0; q < UNR; ++q) {
            ur[q] = *reinterpret_cast<const TV*>(col + (size_t)(k + q) * mp);
            ui[q] = *reinterpret_cast<const TV*>(col + (size_t)(k + q) * mp + plane);
          }
          // state values four at a time (one wide LDS broadcast per four k)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            if (c >= d) break;
#pragma unroll
            for (int q4 = 0; q4 < UNR; q4 += 4) {
              T pr4[4], pi4[4];
              *reinterpret_cast<T4*>(pr4) = *reinterpret_cast<const T4*>(sre + c * mp + k + q4);
              *reinterpret_cast<T4*>(pi4) = *reinterpret_cast<const T4*>(sim + c * mp + k + q4);
#pragma unroll
              for (int e4 = 0; e4 < 4; ++e4) {
                const T* urq = reinterpret_cast<const T*>(&ur[q4 + e4]);
                const T* uiq = reinterpret_cast<const T*>(&ui[q4 + e4]);
#pragma unroll
                for (int t = 0; t < RPL; ++t) {
                  a[c][0][t] += urq[t] * pr4[e4] - uiq[t] * pi4[e4];
                  a[c][1][t] += urq[t] * pi4[e4] + uiq[t] * pr4[e4];
                }
              }
            }
          }
        }
        for (; k < k1; ++k) {
          const TV ur = *reinterpret_cast<const TV*>(col + (size_t)k * mp);
          const TV ui = *reinterpret_cast<const TV*>(col + (size_t)k * mp + plane);
          const T* urq = reinterpret_cast<const T*>(&ur);
          const T* uiq = reinterpret_cast<const T*>(&ui);
          for (int c = 0; c < d; ++c) {
            const T pr = sre[c * mp + k], pi = sim[c * mp + k];
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
              a[c][0][t] += urq[t] * pr - uiq[t] * pi;
              a[c][1][t] += urq[t] * pi + uiq[t] * pr;
            }
          }
        }
      }
      if (i0 < mp) {
        for (int c = 0; c < d; ++c) {
          T* p0 = pre + ((size_t)kg * d + c) * mp + i0;
          T* q0 = pim + ((size_t)kg * d + c) * mp + i0;
#pragma unroll
          for (int t = 0; t < RPL; ++t) {
            p0[t] = a[c][0][t];
            q0[t] = a[c][1][t];
          }
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

// ---- backward sweeps from the forward store.  Row i of U^dag is the conjugate of column i
// of U, contiguous in memory, so each entry of lambda_j = U_j^dag lambda_{j+1} is a dot
// product down one column.  KL lanes share a row; each takes RPL consecutive entries of
// the column (one 16-byte load per plane) per pass of KL * RPL entries, and the KL partial
// sums meet by butterfly shuffles.  Entries at or beyond m are masked (the state is zero
// there and the padding of U is never read into a sum).
template <typename T, int KL, int UNR>
__device__ inline void dag_row_acc(const T* col, size_t plane, int m, int k0, const T* sre, const T* sim, int mp,
                                   int d, T (&a)[2][2]) {
  typedef typename Vec16<T>::type TV;
  constexpr int RPL = Vec16<T>::n, STEP = KL * RPL;
  for (int kb = k0; kb < m; kb += STEP * UNR) {
    TV ur[UNR] = {}, ui[UNR] = {};
#pragma unroll
    for (int q = 0; q < UNR; ++q) {
      const int k = kb + q * STEP;
      if (k < m) {
        ur[q] = *reinterpret_cast<const TV*>(col + k);
        ui[q] = *reinterpret_cast<const TV*>(col + k + plane);
      }
    }
#pragma unroll
    for (int q = 0; q < UNR; ++q) {
      const int k = kb + q * STEP;
      if (k >= m) break;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (c >= d) break;
        const TV pr = *reinterpret_cast<const TV*>(sre + c * mp + k);
        const TV pi = *reinterpret_cast<const TV*>(sim + c * mp + k);
#pragma unroll
        for (int e = 0; e < RPL; ++e) {
          const bool in = k + e < m;
          const T xr = in ? ur[q][e] : T(0), xi = in ? ui[q][e] : T(0);
          // conj(x) p = (xr pr + xi pi) + i (xr pi - xi pr)
          a[c][0] += xr * pr[e] + xi * pi[e];
          a[c][1] += xr * pi[e] - xi * pr[e];
        }
      }
    }
  }
}

// sum over each group of KL consecutive lanes (every lane of the group ends with the total)
template <int KL, typename T>
__device__ inline void lane_group_sum(T (&a)[2][2]) {
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      T v = a[c][h];
#pragma unroll
      for (int sh = 1; sh < KL; sh <<= 1) v += __shfl_xor(v, sh);
      a[c][h] = v;
    }
}

// One work-group sweeps one job backwards through the segment: the 16 waves take the rows
// RW = RPL at a time; the state and the next one alternate between two LDS buffers, so a
// slice costs one barrier.
template <typename T>
__device__ void sweep_solo_bwd(const JobDev& jb, char* ws, size_t off_T, int seg_j0, int seg_len) {
  constexpr int RPL = Vec16<T>::n, RW = RPL, KL = 64 / RW;
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  const int len = job_len(jb, seg_j0, seg_len);
  if (len <= 0) return;
  const int m = jb.m, mp = jb.mp, d = jb.d, N = jb.N;
  T* cre = reinterpret_cast<T*>(smem_raw);  // state [d][mp], then the next state
  T* cim = cre + (size_t)d * mp;
  T* nre = cim + (size_t)d * mp;
  T* nim = nre + (size_t)d * mp;
  T* S = tplane<T>(ws, off_T, jb.lam_off);
  const size_t ps = (size_t)mp * N * d;
  const size_t plane = (size_t)mp * mp;
  {
    const int col_in = seg_j0 + len - 1;
    for (int idx = threadIdx.x; idx < mp * d; idx += blockDim.x) {
      const int c = idx / mp, i = idx % mp;
      const size_t g = ((size_t)col_in * d + c) * mp + i;
      cre[idx] = S[g];
      cim[idx] = S[g + ps];
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int rr = lane / KL, kl = lane % KL;
  for (int it = 0; it < len; ++it) {
    const int jl = len - 1 - it;
    const T* U = entry_U<T>(jb, ws, off_T, jl);
    const int col_out = seg_j0 + jl - 1;
    for (int rg = wave; rg * RW < mp; rg += nw) {
      const int i = rg * RW + rr;  // < mp (a multiple of 16)
      T a[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
      if (i < m) dag_row_acc<T, KL, 4>(U + (size_t)i * mp, plane, m, kl * RPL, cre, cim, mp, d, a);
      lane_group_sum<KL>(a);
      if (kl == 0)
        for (int c = 0; c < d; ++c) {
          nre[c * mp + i] = a[c][0];
          nim[c * mp + i] = a[c][1];
          if (col_out >= 0) {
            const size_t g = ((size_t)col_out * d + c) * mp + i;
            S[g] = a[c][0];
            S[g + ps] = a[c][1];
          }
        }
    }
    __syncthreads();
    T* t = cre;
    cre = nre;
    nre = t;
    t = cim;
    cim = nim;
    nim = t;
  }
}

template <typename T, int DIR>
__global__ void __launch_bounds__(1024) k_sweep(const JobDev* jobs, int njobs, char* ws, size_t off_T,
                                                const int* ent_s, const int* ent_q, int r, int seg_j0, int seg_len) {
  const int J = blockIdx.x;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  if constexpr (DIR == 1)
    sweep_solo_bwd<T>(jb, ws, off_T, seg_j0, seg_len);
  else
    sweep_solo<T, DIR>(jb, ws, off_T, ent_s, ent_q, r, seg_j0, seg_len);
}

// ---- co-operative sweep: the rows of a job are split over W = ceil(mp / RB) work-groups
// (RB = 64 FP32 / 32 FP64 rows).  After every slice each group publishes its rows of the
// new state as tagged 64-bit words (a 32-bit half of a value and the slice number, one
// single-copy-atomic store), into one of two buffers by slice parity; every group reads
// the whole state back, spinning on each word until its tag is the slice it waits for.
// Data and flag travel together, so no fences or counters sit on the per-slice path.  A
// group overwrites the words of slice j - 2 only after reading every group's slice j - 1,
// which each wrote after it had read slice j - 2.  All waits are bounded.  Group 0 first
// waits (bounded) for the other groups to arrive; if they are not all resident it runs the
// job alone (sweep_solo) and the late groups leave, so the sweep never depends on
// co-residency.  Control words per job: [0] arrivals, [1] decision (zeroed before the
// launch, with the exchange words).
constexpr int kCoopGo = 1, kCoopSolo = 2;
constexpr long kArriveSpins = 1L << 15;  // ~ms: group 0 waits this long for the others
constexpr long kStepSpins = 1L << 20;    // a stalled hand-off (tens of ms) aborts the sweep
constexpr int kFlagSweepAbort = 4;       // status bit 2: a co-operative sweep gave up

template <typename T> struct CoopRows { static constexpr int value = 16 * Vec16<T>::n; };

__device__ inline int coop_decide(int* ctl, int W, int* flags, int force_solo) {
  __shared__ int decision;
  if (threadIdx.x == 0) {
    if (W == 1) {
      decision = kCoopGo;
    } else if (blockIdx.x == 0) {
      long s = 0;
      while (!force_solo && __hip_atomic_load(ctl + 0, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < W - 1 &&
             ++s < kArriveSpins)
        __builtin_amdgcn_s_sleep(2);
      const int all = !force_solo && __hip_atomic_load(ctl + 0, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= W - 1;
      // the others read the decision; once written it never changes
      decision = all ? kCoopGo : kCoopSolo;
      __hip_atomic_store(ctl + 1, decision, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_fetch_add(ctl + 0, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      int st = 0;
      long s = 0;
      while ((st = __hip_atomic_load(ctl + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) == 0 && ++s < kStepSpins)
        __builtin_amdgcn_s_sleep(2);
      if (st == 0) __hip_atomic_fetch_or(flags, kFlagSweepAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      decision = st == kCoopGo ? kCoopGo : 0;  // solo or no decision: this group leaves
    }
  }
  __syncthreads();
  return decision;
}

// Tagged exchange words: a 32-bit half of a value in the low word, the tag in the high one.
__device__ inline void xchg_put(unsigned long long* p, unsigned bits, unsigned tag) {
  __hip_atomic_store(p, ((unsigned long long)tag << 32) | bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// spins (bounded) until each of the N words carries tag; false on time-out.  Every load is
// issued before any tag is checked, so one round trip covers all N words.
template <int N>
__device__ inline bool xchg_get_n(const unsigned long long* const (&p)[N], unsigned tag, unsigned (&bits)[N]) {
  unsigned long long w[N];
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] = __hip_atomic_load(p[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  long s = 0;
  for (;;) {
    bool all = true;
#pragma unroll
    for (int i = 0; i < N; ++i) all = all && (unsigned)(w[i] >> 32) == tag;
    if (all) {
#pragma unroll
      for (int i = 0; i < N; ++i) bits[i] = (unsigned)w[i];
      return true;
    }
    if (++s >= kStepSpins) return false;
    __builtin_amdgcn_s_sleep(1);
#pragma unroll
    for (int i = 0; i < N; ++i)
      if ((unsigned)(w[i] >> 32) != tag) w[i] = __hip_atomic_load(p[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}
template <typename T> struct XchgVal;
template <> struct XchgVal<float> {
  static constexpr int W = 1;
  __device__ static void put(unsigned long long* p, float v, unsigned tag) { xchg_put(p, __float_as_uint(v), tag); }
  // the values at a and b (the two planes of one state entry)
  __device__ static bool get_pair(const unsigned long long* a, const unsigned long long* b, unsigned tag, float& va,
                                  float& vb) {
    const unsigned long long* const p[2] = {a, b};
    unsigned w[2];
    if (!xchg_get_n<2>(p, tag, w)) return false;
    va = __uint_as_float(w[0]);
    vb = __uint_as_float(w[1]);
    return true;
  }
};
template <> struct XchgVal<double> {
  static constexpr int W = 2;
  __device__ static void put(unsigned long long* p, double v, unsigned tag) {
    const unsigned long long b = __double_as_longlong(v);
    xchg_put(p, (unsigned)b, tag);
    xchg_put(p + 1, (unsigned)(b >> 32), tag);
  }
  __device__ static bool get_pair(const unsigned long long* a, const unsigned long long* b, unsigned tag, double& va,
                                  double& vb) {
    const unsigned long long* const p[4] = {a, a + 1, b, b + 1};
    unsigned w[4];
    if (!xchg_get_n<4>(p, tag, w)) return false;
    va = __longlong_as_double((long long)(((unsigned long long)w[1] << 32) | w[0]));
    vb = __longlong_as_double((long long)(((unsigned long long)w[3] << 32) | w[2]));
    return true;
  }
};

// A job whose rows fit one work-group (W = 1) needs no exchange: the new state goes straight
// back into LDS, and the next slice's propagator entries (one column segment per lane, as
// every column index k < m <= RB lands in the first column block of a wave) are loaded while
// the current slice is applied, so the per-slice cost is two work-group barriers.  When every
// job of a plan fits one group, the sweep is launched with only the waves the widest block
// needs (4 columns per wave), so the barriers span fewer waves.
template <typename T, int DIR>
__device__ void sweep_single(const JobDev& jb, char* ws, size_t off_T, int seg_j0, int len, char* smem_raw) {
  static_assert(DIR == 0, "the backward one-group sweep is sweep_single_bwd");
  typedef typename Vec16<T>::type TV;
  constexpr int RPL = Vec16<T>::n, RB = CoopRows<T>::value;
  const int m = jb.m, mp = jb.mp, d = jb.d, N = jb.N;
  T* sre = reinterpret_cast<T*>(smem_raw);  // state [d][mp]
  T* sim = sre + (size_t)d * mp;
  T* pre = sim + (size_t)d * mp;             // wave partials [16][d][RB]
  T* pim = pre + (size_t)16 * d * RB;
  T* S = tplane<T>(ws, off_T, DIR == 0 ? jb.psi_off : jb.lam_off);
  const size_t ncol = DIR == 0 ? (size_t)(N + 1) * d : (size_t)N * d;
  const size_t ps = (size_t)mp * ncol;
  const size_t plane = (size_t)mp * mp;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int rv = lane & 15, kk = lane >> 4;
  const int row = rv * RPL, k = 4 * wave + kk;  // rows row .. row + RPL - 1 of column k (4 nw >= m)
  const bool act = row < m && k < m;
  {
    const int col_in = DIR == 0 ? seg_j0 : seg_j0 + len - 1;
    for (int idx = threadIdx.x; idx < mp * d; idx += blockDim.x) {
      const int c = idx / mp, i = idx % mp;
      const size_t g = ((size_t)col_in * d + c) * mp + i;
      sre[idx] = S[g];
      sim[idx] = S[g + ps];
    }
  }
  TV ur = {}, ui = {};
  if (act) {
    const T* U = entry_U<T>(jb, ws, off_T, DIR == 0 ? 0 : len - 1) + row + (size_t)k * mp;
    ur = *reinterpret_cast<const TV*>(U);
    ui = *reinterpret_cast<const TV*>(U + plane);
  }
  __syncthreads();
  for (int it = 0; it < len; ++it) {
    const int jl = DIR == 0 ? it : len - 1 - it;
    TV nr = {}, ni = {};
    if (act && it + 1 < len) {
      const T* U = entry_U<T>(jb, ws, off_T, DIR == 0 ? jl + 1 : jl - 1) + row + (size_t)k * mp;
      nr = *reinterpret_cast<const TV*>(U);
      ni = *reinterpret_cast<const TV*>(U + plane);
    }
    T a[2][2][RPL];  // [copy][re, im][row]
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int t = 0; t < RPL; ++t) a[c][0][t] = a[c][1][t] = T(0);
    if (act) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (c >= d) break;
        const T pr = sre[c * mp + k], pi = sim[c * mp + k];
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          a[c][0][t] = ur[t] * pr - ui[t] * pi;
          a[c][1][t] = ur[t] * pi + ui[t] * pr;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          T v = a[c][h][t];
          v += __shfl_xor(v, 16);
          v += __shfl_xor(v, 32);
          a[c][h][t] = v;
        }
    if (kk == 0)
      for (int c = 0; c < d; ++c)
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          pre[((size_t)wave * d + c) * RB + row + t] = a[c][0][t];
          pim[((size_t)wave * d + c) * RB + row + t] = a[c][1][t];
        }
    __syncthreads();
    const int col_out = DIR == 0 ? seg_j0 + jl + 1 : seg_j0 + jl - 1;
    if ((int)threadIdx.x < RB * d) {
      const int c = threadIdx.x / RB, i = threadIdx.x % RB;
      T vr = T(0), vi = T(0);
      for (int w = 0; w < nw; ++w) {
        vr += pre[((size_t)w * d + c) * RB + i];
        vi += pim[((size_t)w * d + c) * RB + i];
      }
      if (i >= m) vr = vi = T(0);
      if (i < mp) {
        sre[c * mp + i] = vr;
        sim[c * mp + i] = vi;
        if (col_out >= 0) {
          const size_t g = ((size_t)col_out * d + c) * mp + i;
          S[g] = vr;
          S[g + ps] = vi;
        }
      }
    }
    __syncthreads();
    ur = nr;
    ui = ni;
  }
}

// The backward sweep of a job whose rows fit one work-group: wave w takes rows 4w .. 4w+3,
// 16 lanes per row cover the column (16 RPL = RB entries); the next slice's column segment
// is loaded while the current one is applied, and the state alternates between two LDS
// buffers, so a slice costs one barrier.
template <typename T>
__device__ void sweep_single_bwd(const JobDev& jb, char* ws, size_t off_T, int seg_j0, int len, char* smem_raw) {
  typedef typename Vec16<T>::type TV;
  constexpr int RPL = Vec16<T>::n, KL = 16;
  const int m = jb.m, mp = jb.mp, d = jb.d, N = jb.N;
  T* st = reinterpret_cast<T*>(smem_raw);  // [buffer][re, im][d][mp]
  T* S = tplane<T>(ws, off_T, jb.lam_off);
  const size_t ps = (size_t)mp * N * d;
  const size_t plane = (size_t)mp * mp;
  const size_t dm = (size_t)d * mp;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rr = lane / KL, kl = lane % KL;
  const int i = 4 * wave + rr, k = kl * RPL;  // 4 waves per 16 rows cover mp (launch width)
  const bool act = i < m && k < m;
  {
    const int col_in = seg_j0 + len - 1;
    for (int idx = threadIdx.x; idx < mp * d; idx += blockDim.x) {
      const int c = idx / mp, ii = idx % mp;
      const size_t g = ((size_t)col_in * d + c) * mp + ii;
      st[idx] = S[g];
      st[dm + idx] = S[g + ps];
    }
  }
  TV ur = {}, ui = {};
  if (act) {
    const T* U = entry_U<T>(jb, ws, off_T, len - 1) + (size_t)i * mp + k;
    ur = *reinterpret_cast<const TV*>(U);
    ui = *reinterpret_cast<const TV*>(U + plane);
  }
  __syncthreads();
  for (int it = 0; it < len; ++it) {
    const int jl = len - 1 - it;
    TV nr = {}, ni = {};
    if (act && it + 1 < len) {
      const T* U = entry_U<T>(jb, ws, off_T, jl - 1) + (size_t)i * mp + k;
      nr = *reinterpret_cast<const TV*>(U);
      ni = *reinterpret_cast<const TV*>(U + plane);
    }
    const T* cre = st + (size_t)(it & 1) * 2 * dm;
    const T* cim = cre + dm;
    T* nre = st + (size_t)((it + 1) & 1) * 2 * dm;
    T* nim = nre + dm;
    T a[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
    if (act) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (c >= d) break;
        const TV pr = *reinterpret_cast<const TV*>(cre + c * mp + k);
        const TV pi = *reinterpret_cast<const TV*>(cim + c * mp + k);
#pragma unroll
        for (int e = 0; e < RPL; ++e) {
          const bool in = k + e < m;
          const T xr = in ? ur[e] : T(0), xi = in ? ui[e] : T(0);
          a[c][0] += xr * pr[e] + xi * pi[e];
          a[c][1] += xr * pi[e] - xi * pr[e];
        }
      }
    }
    lane_group_sum<KL>(a);
    const int col_out = seg_j0 + jl - 1;
    if (kl == 0 && i < mp)
      for (int c = 0; c < d; ++c) {
        nre[c * mp + i] = a[c][0];
        nim[c * mp + i] = a[c][1];
        if (col_out >= 0) {
          const size_t g = ((size_t)col_out * d + c) * mp + i;
          S[g] = a[c][0];
          S[g + ps] = a[c][1];
        }
      }
    __syncthreads();
    ur = nr;
    ui = ni;
  }
}

// The backward co-operative sweep's slices (after the groups agreed to go): rows of this
// group r0 .. r0 + RB - 1, wave w rows r0 + RW w .. + RW - 1 with KL = 64 / RW lanes each;
// the hand-off is the forward sweep's (tagged words by slice parity).  One LDS state
// buffer: a barrier after each slice keeps the next slice's state read behind every
// wave's use of the current one.
template <typename T>
__device__ void sweep_coop_bwd(const JobDev& jb, char* ws, size_t off_T, int seg_j0, int len,
                               unsigned long long* X, int* flags, unsigned tag_skew, char* smem_raw) {
  typedef XchgVal<T> XV;
  constexpr int RPL = Vec16<T>::n, RB = CoopRows<T>::value, RW = RPL, KL = 64 / RW;
  __shared__ int abort_now;
  const int m = jb.m, mp = jb.mp, d = jb.d, N = jb.N;
  T* sre = reinterpret_cast<T*>(smem_raw);  // state [d][mp]
  T* sim = sre + (size_t)d * mp;
  T* S = tplane<T>(ws, off_T, jb.lam_off);
  const size_t ps = (size_t)mp * N * d;
  const size_t plane = (size_t)mp * mp;
  const size_t xplane = (size_t)d * mp * XV::W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rr = lane / KL, kl = lane % KL;
  const int i = blockIdx.x * RB + wave * RW + rr;
  {
    const int col_in = seg_j0 + len - 1;
    for (int idx = threadIdx.x; idx < mp * d; idx += blockDim.x) {
      const int c = idx / mp, ii = idx % mp;
      const size_t g = ((size_t)col_in * d + c) * mp + ii;
      sre[idx] = S[g];
      sim[idx] = S[g + ps];
    }
    if (threadIdx.x == 0) abort_now = 0;
    __syncthreads();
  }
  for (int it = 0; it < len; ++it) {
    const int jl = len - 1 - it;
    if (it > 0) {
      // the state after slice it - 1, published by every group with tag it
      const unsigned long long* Xp = X + (size_t)((it - 1) & 1) * 2 * xplane;
      bool ok = true;
      for (int idx = threadIdx.x; idx < mp * d && ok; idx += blockDim.x) {
        T vr = T(0), vi = T(0);
        ok = XV::get_pair(Xp + (size_t)idx * XV::W, Xp + xplane + (size_t)idx * XV::W, (unsigned)it + tag_skew, vr,
                          vi);
        sre[idx] = vr;
        sim[idx] = vi;
      }
      if (!ok) {
        abort_now = 1;
        __hip_atomic_fetch_or(flags, kFlagSweepAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
      if (abort_now) return;
    }
    const T* U = entry_U<T>(jb, ws, off_T, jl);
    T a[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
    if (i < m) dag_row_acc<T, KL, 4>(U + (size_t)i * mp, plane, m, kl * RPL, sre, sim, mp, d, a);
    lane_group_sum<KL>(a);
    const int col_out = seg_j0 + jl - 1;
    if (kl == 0 && i < mp)
      for (int c = 0; c < d; ++c) {
        if (it + 1 < len) {
          unsigned long long* Xo = X + (size_t)(it & 1) * 2 * xplane + ((size_t)c * mp + i) * XV::W;
          XV::put(Xo, a[c][0], (unsigned)(it + 1));
          XV::put(Xo + xplane, a[c][1], (unsigned)(it + 1));
        }
        if (col_out >= 0) {
          const size_t g = ((size_t)col_out * d + c) * mp + i;
          S[g] = a[c][0];
          S[g + ps] = a[c][1];
        }
      }
    __syncthreads();
  }
}

// mode (host test switches, 0 in normal use): bit 0 -- group 0 runs every multi-group job
// alone without waiting for the others (sweep_solo); bit 1 -- the groups wait for hand-off
// tags that are never written, so every bounded wait times out and the sweep gives up with
// status bit 2, as it would on a real stall.
template <typename T, int DIR>
__global__ void __launch_bounds__(1024) k_sweep_coop(const JobDev* jobs, int njobs, char* ws, size_t off_T,
                                                     const int* ent_s, const int* ent_q, int r, int seg_j0,
                                                     int seg_len, int* ctl_all, int* flags,
                                                     unsigned long long* xchg_all, int mode) {
  typedef typename Vec16<T>::type TV;
  typedef XchgVal<T> XV;
  constexpr int RPL = Vec16<T>::n, RB = CoopRows<T>::value, UNR = 4;
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  const int J = blockIdx.y;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  const int len = job_len(jb, seg_j0, seg_len);
  if (len <= 0) return;
  const int m = jb.m, mp = jb.mp, d = jb.d, N = jb.N;
  const int W = (mp + RB - 1) / RB;
  if ((int)blockIdx.x >= W) return;
  if (W == 1) {
    if constexpr (DIR == 1)
      sweep_single_bwd<T>(jb, ws, off_T, seg_j0, len, smem_raw);
    else
      sweep_single<T, DIR>(jb, ws, off_T, seg_j0, len, smem_raw);
    return;
  }
  int* ctl = ctl_all + 4 * J;
  const int decision = coop_decide(ctl, W, flags, mode & 1);
  if (decision == kCoopSolo) {
    if constexpr (DIR == 1)
      sweep_solo_bwd<T>(jb, ws, off_T, seg_j0, seg_len);
    else
      sweep_solo<T, DIR>(jb, ws, off_T, ent_s, ent_q, r, seg_j0, seg_len);
    return;
  }
  if (decision != kCoopGo) return;
  // tags run 1 .. len - 1 < 2^24 (N <= 2^24): the skewed tag is never written
  const unsigned tag_skew = (mode & 2) ? (1u << 30) : 0u;
  if (DIR == 1) {
    sweep_coop_bwd<T>(jb, ws, off_T, seg_j0, len, xchg_all + jb.xchg_off, flags, tag_skew, smem_raw);
    return;
  }
  T* sre = reinterpret_cast<T*>(smem_raw);  // state [d][mp]
  T* sim = sre + (size_t)d * mp;
  T* pre = sim + (size_t)d * mp;             // wave partials [16][d][RB]
  T* pim = pre + (size_t)16 * d * RB;
  __shared__ int abort_now;
  T* S = tplane<T>(ws, off_T, DIR == 0 ? jb.psi_off : jb.lam_off);
  const size_t ncol = DIR == 0 ? (size_t)(N + 1) * d : (size_t)N * d;
  const size_t ps = (size_t)mp * ncol;
  const size_t plane = (size_t)mp * mp;
  // exchange words of this job: [parity][re, im][d][mp] values of XV::W words
  unsigned long long* X = xchg_all + jb.xchg_off;
  const size_t xplane = (size_t)d * mp * XV::W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rv = lane & 15, kk = lane >> 4;
  const int r0 = blockIdx.x * RB, row = r0 + rv * RPL;  // this lane's rows row .. row + RPL - 1
  const int KC = ((m + 15) / 16 + 3) / 4 * 4;           // columns per wave (multiple of 4)
  const int kw0 = wave * KC, kw1 = min(m, kw0 + KC);
  // the input state of the first slice (written before the launch)
  {
    const int col_in = DIR == 0 ? seg_j0 : seg_j0 + len - 1;
    for (int idx = threadIdx.x; idx < mp * d; idx += blockDim.x) {
      const int c = idx / mp, i = idx % mp;
      const size_t g = ((size_t)col_in * d + c) * mp + i;
      sre[idx] = S[g];
      sim[idx] = S[g + ps];
    }
    if (threadIdx.x == 0) abort_now = 0;
    __syncthreads();
  }
  for (int it = 0; it < len; ++it) {
    const int jl = DIR == 0 ? it : len - 1 - it;
    if (it > 0) {
      // the state after slice it - 1, published by every group with tag it
      const unsigned long long* Xp = X + (size_t)((it - 1) & 1) * 2 * xplane;
      bool ok = true;
      for (int idx = threadIdx.x; idx < mp * d && ok; idx += blockDim.x) {
        T vr = T(0), vi = T(0);
        ok = XV::get_pair(Xp + (size_t)idx * XV::W, Xp + xplane + (size_t)idx * XV::W, (unsigned)it + tag_skew, vr,
                          vi);
        sre[idx] = vr;
        sim[idx] = vi;
      }
      if (!ok) {
        abort_now = 1;
        __hip_atomic_fetch_or(flags, kFlagSweepAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
      if (abort_now) return;
    }
    const T* U = entry_U<T>(jb, ws, off_T, jl);
    T a[2][2][RPL];  // [copy][re, im][row]
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int t = 0; t < RPL; ++t) a[c][0][t] = a[c][1][t] = T(0);
    if (row < m) {
      for (int kb = kw0; kb < kw1; kb += 4 * UNR) {
        TV ur[UNR], ui[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int k = kb + 4 * u + kk;
          if (k < kw1) {
            ur[u] = *reinterpret_cast<const TV*>(U + row + (size_t)k * mp);
            ui[u] = *reinterpret_cast<const TV*>(U + row + (size_t)k * mp + plane);
          }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int k = kb + 4 * u + kk;
          if (k >= kw1) break;
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            if (c >= d) break;
            const T pr = sre[c * mp + k], pi = sim[c * mp + k];
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
              a[c][0][t] += ur[u][t] * pr - ui[u][t] * pi;
              a[c][1][t] += ur[u][t] * pi + ui[u][t] * pr;
            }
          }
        }
      }
    }
    // sum the four column phases of the wave, then the 16 waves
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          T v = a[c][h][t];
          v += __shfl_xor(v, 16);
          v += __shfl_xor(v, 32);
          a[c][h][t] = v;
        }
    if (kk == 0)
      for (int c = 0; c < d; ++c)
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          pre[((size_t)wave * d + c) * RB + rv * RPL + t] = a[c][0][t];
          pim[((size_t)wave * d + c) * RB + rv * RPL + t] = a[c][1][t];
        }
    __syncthreads();
    const int col_out = DIR == 0 ? seg_j0 + jl + 1 : seg_j0 + jl - 1;
    if ((int)threadIdx.x < RB * d) {
      const int c = threadIdx.x / RB, i = threadIdx.x % RB;
      T vr = T(0), vi = T(0);
      for (int w = 0; w < 16; ++w) {
        vr += pre[((size_t)w * d + c) * RB + i];
        vi += pim[((size_t)w * d + c) * RB + i];
      }
      if (r0 + i >= m) vr = vi = T(0);
      if (r0 + i < mp) {
        if (it + 1 < len) {
          unsigned long long* Xo = X + (size_t)(it & 1) * 2 * xplane + ((size_t)c * mp + r0 + i) * XV::W;
          XV::put(Xo, vr, (unsigned)(it + 1));
          XV::put(Xo + xplane, vi, (unsigned)(it + 1));
        }
        if (col_out >= 0) {
          const size_t g = ((size_t)col_out * d + c) * mp + r0 + i;
          S[g] = vr;
          S[g + ps] = vi;
        }
      }
    }
    // no barrier here: the next slice's state read ends with one before the partials are
    // written again, and this slice's reads of the state in LDS are behind the one above
  }
}

// ===================================================================== objective
// Per problem (one work-group each): o = sum <psi_f|psi_N>, ||psi_N||^2, ||psi_f||^2 in
// FP64 with a fixed-order reduction.
template <typename T>
__global__ void __launch_bounds__(1024) k_overlap(const JobDev* jobs, const ProbDev* probs, char* ws, size_t off_T,
                                                  const int* flags, double* out) {
  __shared__ double red[4][1024];
  const ProbDev pb = probs[blockIdx.x];
  double o_r = 0.0, o_i = 0.0, nn = 0.0, nf = 0.0;
  for (int J = pb.job_begin; J < pb.job_end; ++J) {
    const JobDev jb = jobs[J];
    const int N = jb.N;
    const T* Pp = tplane<T>(ws, off_T, jb.psi_off);
    const T* Lm = tplane<T>(ws, off_T, jb.lam_off);
    const size_t pps = (size_t)jb.mp * (N + 1) * jb.d, lps = (size_t)jb.mp * N * jb.d;
    for (int idx = threadIdx.x; idx < jb.m * jb.d; idx += blockDim.x) {
      const int c = idx / jb.m, i = idx % jb.m;
      const size_t gp = ((size_t)N * jb.d + c) * jb.mp + i;
      const size_t gl = ((size_t)(N - 1) * jb.d + c) * jb.mp + i;
      const double pr = Pp[gp], pi = Pp[gp + pps], fr = Lm[gl], fi = Lm[gl + lps];
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
    double* o = out + (size_t)blockIdx.x * 8;
    const double orr = red[0][0], oii = red[1][0], nN = red[2][0], nF = red[3][0];
    const double raw = orr * orr + oii * oii;
    o[0] = raw / (nN * nF);
    o[1] = raw;
    o[2] = orr;
    o[3] = oii;
    o[4] = nN;
    o[5] = nF;
    int fl = flags[0];
    if (!isfinite(o[0])) fl |= 2;
    o[6] = (double)flags[1];
    o[7] = (double)fl;
  }
}

// ===================================================================== gradient series
// Z_o = H_o * V for every (job, o); V and Z are gradient slots of the job.
template <typename Shape>
__global__ void __launch_bounds__(256, Shape::WAVES)
    k_panel_gemm(const JobDev* jobs, const PanelDesc* descs, int ndesc, long long total_items, char* ws,
                 size_t off_T, int vslot, int j0) {
  typedef typename Shape::T T;
  __shared__ TileSmem<Shape> lds;
  const ItemRange rg = xcd_items(total_items);
  ItemCursor cur;
  struct Item {
    TileOperands<T> op;
    T* C;
    long long vplane;
  };
  auto prep = [&](long long it, Item& x) -> bool {
    const PanelDesc pd = descs[cursor_find(descs, ndesc, it, cur)];
    const JobDev jb = jobs[pd.job];
    if (jb.N - j0 <= 0) return false;
    const long long local = it - pd.item_off;
    const int ti = (int)(local / pd.tiles_n), tj = (int)(local % pd.tiles_n);
    const int mp = jb.mp;
    const size_t hplane = (size_t)mp * mp;
    const size_t vplane = (size_t)mp * jb.cc;
    T* g = tplane<T>(ws, off_T, jb.gbase_off);
    x.op.A = reinterpret_cast<const T*>(jb.hT) + (size_t)(2 * pd.op) * hplane;
    x.op.a_ps = hplane;
    x.op.lda = mp;
    x.op.B = g + (size_t)vslot * jb.gslot;
    x.op.b_ps = vplane;
    x.op.ldb = mp;
    x.op.M = mp;
    x.op.N = jb.cc;
    x.op.K = mp;
    x.op.row0 = ti * Shape::BM;
    x.op.col0 = tj * Shape::BN;
    x.C = g + (size_t)pd.op * jb.gslot;
    x.vplane = (long long)vplane;
    return true;
  };
  long long it = rg.begin;
  Item x;
  while (it < rg.end && !prep(it, x)) it += rg.step;
  if (it >= rg.end) return;
  TilePipe pipe = tile_start<Shape>(x.op, lds);
  for (;;) {
    long long nx = it + rg.step;
    Item xn = x;
    while (nx < rg.end && !prep(nx, xn)) nx += rg.step;
    const bool more = nx < rg.end;
    TileAcc<Shape> acc;
    tile_mma<Shape>(x.op, lds, acc, pipe, more, xn.op);
    const int mp = x.op.M;
#pragma unroll
    for (int ri = 0; ri < Shape::SM; ++ri)
#pragma unroll
      for (int ci = 0; ci < Shape::SN; ++ci) {
        const int rbase = acc_row_base<Shape>(x.op.row0, ri);
        const int col = acc_col<Shape>(x.op.col0, ci);
        if (rbase >= mp || col >= x.op.N) continue;
        T* cr = x.C + (size_t)(rbase + acc_row_off<T>(0)) + (size_t)col * mp;
        acc_store<T>(cr, acc.re[ri][ci]);
        acc_store<T>(cr + x.vplane, acc.im[ri][ci]);
      }
    if (!more) break;
    it = nx;
    x = xn;
  }
}

// ===================================================================== operator products
// C = A B, or C += A B, for square mp x mp complex blocks (planar, column-major), on the
// matrix cores with the propagator GEMM's tile: the operator products, once per system
// (ensure_powers, FP64) or at the start of each call into the workspace
// (Driver::form_products, the working precision).  An operand whose bit is set in `rel`
// (1 A, 2 B, 4 C) holds a byte offset from the kernel's `base` (the workspace) instead of
// an address.
template <typename T>
struct SetupGemmT {
  const T* A;
  const T* B;
  T* C;
  long long item_off;
  int mp, tiles_n, accumulate, rel;
};

// The set-up GEMM tile that forms workspace products in a plan's precision.
template <typename T> struct ProductShape;
template <> struct ProductShape<float> { typedef TileShape<float, 2, 2, 2> type; };
template <> struct ProductShape<double> { typedef TileShape<double, 2, 2, 2> type; };

template <typename T>
__device__ inline T* rel_ptr(const T* p, int is_rel, char* base) {
  T* q = is_rel ? reinterpret_cast<T*>(base + reinterpret_cast<uintptr_t>(p)) : const_cast<T*>(p);
  return global_ptr(q);
}

template <typename Shape>
__global__ void __launch_bounds__(256, Shape::WAVES)
    k_setup_gemm(const SetupGemmT<typename Shape::T>* descs, int ndesc, long long total_items, char* base) {
  typedef typename Shape::T T;
  __shared__ TileSmem<Shape> lds;
  const ItemRange rg = xcd_items(total_items);
  ItemCursor cur;
  struct Item {
    TileOperands<T> op;
    T* C;
    int accumulate;
  };
  auto prep = [&](long long it, Item& x) -> bool {
    const SetupGemmT<T> g = descs[cursor_find(descs, ndesc, it, cur)];
    const long long local = it - g.item_off;
    const size_t plane = (size_t)g.mp * g.mp;
    x.op.A = rel_ptr(g.A, g.rel & 1, base);
    x.op.a_ps = plane;
    x.op.lda = g.mp;
    x.op.B = rel_ptr(g.B, g.rel & 2, base);
    x.op.b_ps = plane;
    x.op.ldb = g.mp;
    x.op.M = g.mp;
    x.op.N = g.mp;
    x.op.K = g.mp;
    x.op.row0 = (int)(local / g.tiles_n) * Shape::BM;
    x.op.col0 = (int)(local % g.tiles_n) * Shape::BN;
    x.C = rel_ptr(g.C, g.rel & 4, base);
    x.accumulate = g.accumulate;
    return true;
  };
  long long it = rg.begin;
  if (it >= rg.end) return;
  Item x;
  prep(it, x);
  TilePipe pipe = tile_start<Shape>(x.op, lds);
  for (;;) {
    const long long nx = it + rg.step;
    Item xn = x;
    const bool more = nx < rg.end;
    if (more) prep(nx, xn);
    TileAcc<Shape> acc;
    tile_mma<Shape>(x.op, lds, acc, pipe, more, xn.op);
    const int mp = x.op.M;
    const size_t plane = (size_t)mp * mp;
#pragma unroll
    for (int ri = 0; ri < Shape::SM; ++ri)
#pragma unroll
      for (int ci = 0; ci < Shape::SN; ++ci) {
        const int rbase = acc_row_base<Shape>(x.op.row0, ri);
        const int col = acc_col<Shape>(x.op.col0, ci);
        if (rbase >= mp || col >= mp) continue;
        T* c = x.C + (size_t)(rbase + acc_row_off<T>(0)) + (size_t)col * mp;
        typename Vec4<T>::type vr = acc.re[ri][ci], vi = acc.im[ri][ci];
        if (x.accumulate) {
          vr += acc_load<T>(c);
          vi += acc_load<T>(c + plane);
        }
        acc_store<T>(c, vr);
        acc_store<T>(c + plane, vi);
      }
    if (!more) break;
    it = nx;
    x = xn;
  }
}

// The product launches of one block (operators H, products PW; either may be a workspace
// byte offset, flagged in rel_h / rel_pw), appended to the five passes, which run in order:
// pass 0 S_ab = H_a H_b (a <= b, lexicographic), pass 1 S_ab += H_b H_a (a < b), passes
// 2..4 the first, second and third term of each triple product, a sum of H_x S_yz over the
// representatives of its distinct orderings: T_aaa = H_a S_aa; T_aac = H_a S_ac + H_c S_aa;
// T_acc = H_a S_cc + H_c S_ac; T_abc = H_a S_bc + H_b S_ac + H_c S_ab (a < b < c).  Item
// offsets run on within each pass.
template <typename T>
static void product_descs(const T* H, int rel_h, T* PW, int rel_pw, int K, int mp, int bm, int bn,
                          std::vector<SetupGemmT<T>> (&pass)[5], long long (&items)[5]) {
  const int O = K + 1;
  const size_t plane = (size_t)mp * mp;
  const int tm = (mp + bm - 1) / bm, tn = (mp + bn - 1) / bn;
  auto op = [&](int o) { return H + (size_t)(2 * o) * plane; };
  auto pw = [&](int idx) { return PW + (size_t)(2 * idx) * plane; };
  auto pair_index = [&](int a, int b) {  // position of (a <= b) in lexicographic order
    int idx = 0;
    for (int x = 0; x < a; ++x) idx += O - x;
    return idx + (b - a);
  };
  auto add = [&](int p, const T* A, int ra, const T* B, int rb, T* C, int acc) {
    pass[p].push_back(SetupGemmT<T>{A, B, C, items[p], mp, tn, acc, (ra ? 1 : 0) | (rb ? 2 : 0) | (rel_pw ? 4 : 0)});
    items[p] += (long long)tm * tn;
  };
  for (int a = 0; a < O; ++a)
    for (int b = a; b < O; ++b) {
      add(0, op(a), rel_h, op(b), rel_h, pw(pair_index(a, b)), 0);
      if (b != a) add(1, op(b), rel_h, op(a), rel_h, pw(pair_index(a, b)), 1);
    }
  int t = pair_count(K);
  for (int a = 0; a < O; ++a)
    for (int b = a; b < O; ++b)
      for (int c = b; c < O; ++c, ++t) {
        std::vector<std::pair<int, int>> terms;  // (x, pair index of the other two)
        if (a == b && b == c) {
          terms = {{a, pair_index(a, a)}};
        } else if (a == b) {
          terms = {{a, pair_index(a, c)}, {c, pair_index(a, a)}};
        } else if (b == c) {
          terms = {{a, pair_index(b, b)}, {b, pair_index(a, b)}};
        } else {
          terms = {{a, pair_index(b, c)}, {b, pair_index(a, c)}, {c, pair_index(a, b)}};
        }
        for (size_t i = 0; i < terms.size(); ++i)
          add(2 + (int)i, op(terms[i].first), rel_h, pw(terms[i].second), rel_pw, pw(t), i > 0 ? 1 : 0);
      }
}

__global__ void k_planes_to_float(const double* a, float* c, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    c[i] = (float)a[i];
}

// Load a chunk of forward states (src = 0) or costates (src = 1) into a gradient slot.
template <typename T>
__global__ void k_chunk_load(const JobDev* jobs, int njobs, char* ws, size_t off_T, int src, int slot, int j0,
                             int chunk) {
  for (int J = blockIdx.y; J < njobs; J += gridDim.y) {
  const JobDev jb = jobs[J];
  const int nsl = min(chunk, jb.N - j0);
  if (nsl <= 0) continue;
  const int mp = jb.mp, d = jb.d, N = jb.N;
  T* g = tplane<T>(ws, off_T, jb.gbase_off) + (size_t)slot * jb.gslot;
  const size_t vplane = (size_t)mp * jb.cc;
  const T* S = tplane<T>(ws, off_T, src == 0 ? jb.psi_off : jb.lam_off);
  const size_t sps = (size_t)mp * (src == 0 ? (size_t)(N + 1) * d : (size_t)N * d);
  const int total = mp * jb.cc;  // < 2^31 (mp <= 4096, cc <= 2 * 2048 + 15)
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    const int col = idx / mp, i = idx - col * mp;
    const int jj = d == 1 ? col : col >> 1, c = d == 1 ? 0 : col & 1;  // d is 1 or 2
    T vr = T(0), vi = T(0);
    if (jj < nsl) {
      const size_t gs = ((size_t)(j0 + jj) * d + c) * mp + i;
      vr = S[gs];
      vi = S[gs + sps];
    }
    g[idx] = vr;
    g[idx + vplane] = vi;
  }
  }
}

// next = (sign i) (dt_J / R) / (t+1) (Z_0 + sum_k u[j,k] Z_k); optionally acc += next
template <typename T>
__global__ void k_series_combine(const JobDev* jobs, int njobs, char* ws, size_t off_T, const double* u, int j0,
                                 int chunk, double sign_over, int R, int out_slot, int acc_slot) {
  for (int J = blockIdx.y; J < njobs; J += gridDim.y) {
  const JobDev jb = jobs[J];
  const int nsl = min(chunk, jb.N - j0);
  if (nsl <= 0) continue;
  const int mp = jb.mp, d = jb.d, K = jb.K;
  const double* uj = u + jb.u_off;
  T* g = tplane<T>(ws, off_T, jb.gbase_off);
  const size_t vplane = (size_t)mp * jb.cc;
  const int total = mp * jb.cc;  // < 2^31 (mp <= 4096, cc <= 2 * 2048 + 15)
  const T cf = (T)(sign_over * jb.dt / R);
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    const int col = idx / mp;
    const int jj = d == 1 ? col : col >> 1;  // d is 1 or 2
    T sr = g[idx], si = g[idx + vplane];  // Z_0
    if (jj < nsl) {
      for (int k = 1; k <= K; ++k) {
        const T uk = (T)uj[(size_t)(j0 + jj) * K + (k - 1)];
        sr += uk * g[(size_t)k * jb.gslot + idx];
        si += uk * g[(size_t)k * jb.gslot + idx + vplane];
      }
    } else {
      sr = si = T(0);
    }
    // (i c) * (sr + i si) = -c si + i c sr
    const T nr = -cf * si, ni = cf * sr;
    T* o = g + (size_t)out_slot * jb.gslot;
    o[idx] = nr;
    o[idx + vplane] = ni;
    if (acc_slot >= 0) {
      T* a = g + (size_t)acc_slot * jb.gslot;
      a[idx] += nr;
      a[idx + vplane] += ni;
    }
  }
  }
}

// G[col][k] += sum_{i < nb} w_{i,t} <b_i | Z_k>, FP64; one wave per (job, column).  The
// weights are real, so this is <sum_i w_i b_i | Z_k>: one pass over the rows forms the
// combined bank vector and its products with up to KG controls at a time (KG = 2 for plans
// with at most two controls: fewer registers, more resident waves; the same sums).
template <typename T, int KG>
__global__ void __launch_bounds__(256) k_series_dot(const JobDev* jobs, int njobs, char* ws, size_t off_T,
                                                    size_t off_gacc, int bank_slot, int nb, const double* w,
                                                    int zero_first, int j0) {
  for (int J = blockIdx.y; J < njobs; J += gridDim.y) {
  const JobDev jb = jobs[J];
  if (jb.N - j0 <= 0) continue;
  const int lane = threadIdx.x & 63;
  for (int col = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); col < jb.cc;
       col += gridDim.x * (blockDim.x >> 6)) {
  const int mp = jb.mp, K = jb.K;
  const T* g = tplane<T>(ws, off_T, jb.gbase_off);
  const size_t vplane = (size_t)mp * jb.cc;
  double2* G = reinterpret_cast<double2*>(ws + off_gacc) + jb.gacc_off + (size_t)col * K;
  const T* Bc = g + (size_t)bank_slot * jb.gslot + (size_t)col * mp;
  for (int k0 = 1; k0 <= K; k0 += KG) {
    const int nk = min(KG, K - k0 + 1);
    double pr[KG], pi[KG];
#pragma unroll
    for (int q = 0; q < KG; ++q) pr[q] = pi[q] = 0.0;
    for (int row = lane; row < jb.m; row += 64) {
      double cr = 0.0, ci = 0.0;
      for (int i = 0; i < nb; ++i) {
        const T* Bv = Bc + (size_t)i * jb.gslot;
        cr += w[i] * (double)Bv[row];
        ci += w[i] * (double)Bv[row + vplane];
      }
#pragma unroll
      for (int q = 0; q < KG; ++q) {
        if (q >= nk) break;
        const T* Z = g + (size_t)(k0 + q) * jb.gslot + (size_t)col * mp;
        const double zr = Z[row], zi = Z[row + vplane];
        pr[q] += cr * zr + ci * zi;
        pi[q] += cr * zi - ci * zr;
      }
    }
#pragma unroll
    for (int q = 0; q < KG; ++q) {
      if (q >= nk) break;
      const double ar = warp_sum(pr[q]), ai = warp_sum(pi[q]);
      if (lane == 0) {
        const int k = k0 + q;
        double2 prev = zero_first ? make_double2(0.0, 0.0) : G[k - 1];
        G[k - 1] = make_double2(prev.x + ar, prev.y + ai);
      }
    }
  }
  }
  }
}

// The whole Frechet series of one (job, slice, copy) in one wave, for plans whose blocks
// are at most 32 wide: lane = row, vectors broadcast through LDS, the operators read
// from the working-precision planes (L2-resident, shared by every slice of a job).  It
// computes what the panel-GEMM route computes term by term: the b-series
// b_0 = lambda^(r), b_{i+1} = +i (dt/R) H_j b_i / (i+1), lambda^(r-1) = sum_i b_i, folded
// at once into c_t^(r) = sum_{i <= Q-1-t} w(t, i) b_i (w = i! t! / (i+t+1)!); then the
// a-series a_0 = psi^(r), a_{t+1} = -i (dt/R) H_j a_t / (t+1), psi^(r+1) = sum_t a_t, with
// G[k] += <c_t^(r)| H_k a_t> in FP64.  One launch replaces the 4 R Q launches of that
// route, which dominate the step for small blocks.
constexpr int kSmallGradRows = 64;
constexpr int kSmallGradMaxRQ = 48;
// up to this width the one-wave series beats the panel-GEMM route (each lane walks m
// columns per product, so the wave's latency grows with m)
constexpr int kSmallGradMaxWidth = 32;

template <typename T>
__device__ inline double2 small_hv(const T* H, size_t hplane, int mp, int m, int row, int o, const T* vr,
                                   const T* vi) {
  T ar = T(0), ai = T(0);
  if (row < m) {
    const T* hr = H + (size_t)(2 * o) * hplane + row;  // global or LDS (staged)
    const T* hi = H + (size_t)(2 * o + 1) * hplane + row;
    for (int c = 0; c < m; ++c) {
      const T xr = hr[(size_t)c * mp], xi = hi[(size_t)c * mp], yr = vr[c], yi = vi[c];
      ar += xr * yr - xi * yi;
      ai += xr * yi + xi * yr;
    }
  }
  return make_double2((double)ar, (double)ai);
}

template <typename T>
__global__ void __launch_bounds__(64) k_grad_small(const JobDev* jobs, int njobs, char* ws, size_t off_T,
                                                   size_t off_gacc, const double* u, const double* w, int R, int Q,
                                                   int j0, int chunk, int hstage) {
  extern __shared__ double cbuf[];  // c_t^(r): [R][Q][64] complex (re, im), then the staged operators
  __shared__ T vr[kSmallGradRows], vi[kSmallGradRows];
  const int J = blockIdx.y;
  if (J >= njobs) return;
  const JobDev jb = jobs[J];
  const int nsl = min(chunk, jb.N - j0);
  const int col = blockIdx.x;  // chunk column: slice jj, copy c
  if (nsl <= 0 || col >= nsl * jb.d) return;
  const int jj = col / jb.d, cp = col % jb.d;
  const int m = jb.m, mp = jb.mp, d = jb.d, N = jb.N, K = jb.K;
  const int row = threadIdx.x;
  const size_t hplane = (size_t)mp * mp;
  const T* H = static_cast<const T*>(jb.hT);
  if (hstage) {  // the block's operator planes fit in LDS: every product reads them there
    T* Hs = reinterpret_cast<T*>(cbuf + (size_t)R * Q * kSmallGradRows * 2);
    for (size_t e = row; e < (size_t)(K + 1) * 2 * hplane; e += kSmallGradRows) Hs[e] = H[e];
    H = Hs;
    __syncthreads();
  }
  const double* uj = u + jb.u_off + (size_t)(j0 + jj) * K;
  const T cdt = (T)(jb.dt / R);
  // H_j v for the vector in (vr, vi), this lane's row, in the working precision
  auto hjv = [&](T& outr, T& outi) {
    T ar = T(0), ai = T(0);
    for (int o = 0; o <= K; ++o) {
      const double2 z = small_hv<T>(H, hplane, mp, m, row, o, vr, vi);
      const T uo = o == 0 ? T(1) : (T)uj[o - 1];
      ar += uo * (T)z.x;
      ai += uo * (T)z.y;
    }
    outr = ar;
    outi = ai;
  };
  // costate lambda_{j+1} and state psi_j of this column
  const T* Lm = tplane<T>(ws, off_T, jb.lam_off);
  const size_t lps = (size_t)mp * N * d;
  const T* Ps = tplane<T>(ws, off_T, jb.psi_off);
  const size_t pps = (size_t)mp * (N + 1) * d;
  const size_t gcol = ((size_t)(j0 + jj) * d + cp) * mp;
  T br = row < m ? Lm[gcol + row] : T(0), bi = row < m ? Lm[gcol + row + lps] : T(0);
  double* C = cbuf;  // index ((r * Q + t) * 64 + row) * 2
  for (int r = R - 1; r >= 0; --r) {
    T sr = br, si = bi;
    for (int t = 0; t < Q; ++t) {
      double* ct = C + ((size_t)(r * Q + t) * kSmallGradRows + row) * 2;
      ct[0] = w[(size_t)t * Q] * (double)br;
      ct[1] = w[(size_t)t * Q] * (double)bi;
    }
    for (int i = 0; i + 1 < Q; ++i) {
      vr[row] = br;
      vi[row] = bi;
      __syncthreads();
      T hr, hi;
      hjv(hr, hi);
      __syncthreads();
      const T cf = cdt / (T)(i + 1);
      br = -cf * hi;  // (+i cf)(hr + i hi)
      bi = cf * hr;
      if (row >= m) br = bi = T(0);
      sr += br;
      si += bi;
      for (int t = 0; t + i + 1 < Q; ++t) {
        double* ct = C + ((size_t)(r * Q + t) * kSmallGradRows + row) * 2;
        const double wt = w[(size_t)t * Q + i + 1];
        ct[0] += wt * (double)br;
        ct[1] += wt * (double)bi;
      }
    }
    br = sr;
    bi = si;
  }
  // a-series and the dots (wave sums; lane 0 keeps the totals in LDS)
  __shared__ double gsum[2 * kMaxControls];
  if (row < 2 * K) gsum[row] = 0.0;
  T ar_ = row < m ? Ps[gcol + row] : T(0), ai_ = row < m ? Ps[gcol + row + pps] : T(0);
  for (int r = 0; r < R; ++r) {
    const bool next_state = r + 1 < R;
    T sr = ar_, si = ai_;
    for (int t = 0; t < Q; ++t) {
      vr[row] = ar_;
      vi[row] = ai_;
      __syncthreads();
      const double* ct = C + ((size_t)(r * Q + t) * kSmallGradRows + row) * 2;
      const double cr = row < m ? ct[0] : 0.0, ci = row < m ? ct[1] : 0.0;
      T hr = T(0), hi = T(0);
      for (int o = 0; o <= K; ++o) {
        const double2 z = small_hv<T>(H, hplane, mp, m, row, o, vr, vi);
        const T uo = o == 0 ? T(1) : (T)uj[o - 1];
        hr += uo * (T)z.x;
        hi += uo * (T)z.y;
        if (o > 0) {
          const double dr = warp_sum(cr * z.x + ci * z.y), di = warp_sum(cr * z.y - ci * z.x);
          if (row == 0) {
            gsum[2 * (o - 1)] += dr;
            gsum[2 * (o - 1) + 1] += di;
          }
        }
      }
      __syncthreads();
      if (t + 1 < Q || next_state) {
        const T cf = cdt / (T)(t + 1);
        ar_ = cf * hi;  // (-i cf)(hr + i hi)
        ai_ = -cf * hr;
        if (row >= m) ar_ = ai_ = T(0);
        sr += ar_;
        si += ai_;
      }
    }
    ar_ = sr;
    ai_ = si;
  }
  __syncthreads();
  double2* G = reinterpret_cast<double2*>(ws + off_gacc) + jb.gacc_off + (size_t)col * K;
  if (row < K) G[row] = make_double2(gsum[2 * row], gsum[2 * row + 1]);
}

// grad[j][k] = 2 Re(conj(o) (-i dt/R) sum_{jobs,copies} G) / (||psi_N||^2 ||psi_f||^2), per problem
__global__ void k_grad_finish(const JobDev* jobs, const ProbDev* probs, const char* ws, size_t off_gacc, int j0,
                              int chunk, int R, const double* out, double* grad) {
  const ProbDev pb = probs[blockIdx.y];
  const int nsl = min(chunk, pb.N - j0);
  const int K = pb.K;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (nsl <= 0 || idx >= nsl * K) return;
  const int jj = idx / K, k = idx % K;
  double sr = 0.0, si = 0.0;
  for (int J = pb.job_begin; J < pb.job_end; ++J) {
    const JobDev jb = jobs[J];
    const double2* G = reinterpret_cast<const double2*>(ws + off_gacc) + jb.gacc_off;
    for (int c = 0; c < jb.d; ++c) {
      const double2 v = G[(size_t)(jj * jb.d + c) * K + k];
      sr += v.x;
      si += v.y;
    }
  }
  const double a = pb.dt / R;
  // (-i a)(sr + i si) = a si - i a sr
  const double dr = a * si, di = -a * sr;
  const double* o = out + (size_t)blockIdx.y * 8;
  const double re = o[2] * dr + o[3] * di;  // Re(conj(o) * d)
  grad[pb.u_off + (size_t)(j0 + jj) * K + k] = 2.0 * re / (o[4] * o[5]);
}

// ===================================================================== gate propagation
// The time-ordered product K = U_{N-1} ... U_1 U_0 of every block (the unitary a pulse
// implements, Sec. III B), as a balanced tree of batched complex GEMMs: at each level,
// factor pair p (slots 2p and 2p+1 of half `src` of the propagator store: half 0 holds U,
// half 1 is room the plan keeps for this tree when it fits) becomes U_{2p+1} U_{2p} in slot
// p of the other half, and an odd last factor is carried over.  The level's items are laid out as
// the propagator GEMM's (echunk pair slots x tiles per job); a launch covers pairs
// c0 .. c0 + echunk - 1.  Reads and writes of one level touch different halves.
template <typename Shape>
__global__ void __launch_bounds__(256, Shape::WAVES)
    k_chain_step(const JobDev* jobs, int njobs, long long total_items, char* ws, size_t off_T, int src, int c0,
                 int npairs) {
  typedef typename Shape::T T;
  __shared__ TileSmem<Shape> lds;
  const ItemRange rg = xcd_items(total_items);
  ItemCursor cur;
  struct Item {
    TileOperands<T> op;
    T* C;
  };
  auto prep = [&](long long it, Item& x) -> bool {
    const int J = cursor_find(jobs, njobs, it, cur);
    const JobDev jb = jobs[J];
    const long long local = it - jb.item_off;
    const int t2 = jb.tiles_m * jb.tiles_n;
    const int p = c0 + (int)(local / t2);
    if (p >= npairs) return false;
    const int tile = (int)(local % t2);
    const int ti = tile / jb.tiles_n, tj = tile % jb.tiles_n;
    const int mp = jb.mp;
    const size_t plane = (size_t)mp * mp;
    T* ub = tplane<T>(ws, off_T, jb.ubuf_off);
    x.op.A = ub + (size_t)(2 * p + 1) * jb.uslot + (size_t)src * 2 * plane;
    x.op.a_ps = plane;
    x.op.lda = mp;
    x.op.B = ub + (size_t)(2 * p) * jb.uslot + (size_t)src * 2 * plane;
    x.op.b_ps = plane;
    x.op.ldb = mp;
    x.op.M = mp;
    x.op.N = mp;
    x.op.K = mp;
    x.op.row0 = ti * Shape::BM;
    x.op.col0 = tj * Shape::BN;
    x.C = ub + (size_t)p * jb.uslot + (size_t)(1 - src) * 2 * plane;
    return true;
  };
  long long it = rg.begin;
  Item x;
  while (it < rg.end && !prep(it, x)) it += rg.step;
  if (it >= rg.end) return;
  TilePipe pipe = tile_start<Shape>(x.op, lds);
  for (;;) {
    long long nx = it + rg.step;
    Item xn = x;
    while (nx < rg.end && !prep(nx, xn)) nx += rg.step;
    const bool more = nx < rg.end;
    TileAcc<Shape> acc;
    tile_mma<Shape>(x.op, lds, acc, pipe, more, xn.op);
    const int mp = x.op.M;
    const size_t plane = (size_t)mp * mp;
#pragma unroll
    for (int ri = 0; ri < Shape::SM; ++ri)
#pragma unroll
      for (int ci = 0; ci < Shape::SN; ++ci) {
        const int rbase = acc_row_base<Shape>(x.op.row0, ri);
        const int col = acc_col<Shape>(x.op.col0, ci);
        if (rbase >= mp || col >= mp) continue;
        T* cr = x.C + (size_t)(rbase + acc_row_off<T>(0)) + (size_t)col * mp;
        acc_store<T>(cr, acc.re[ri][ci]);
        acc_store<T>(cr + plane, acc.im[ri][ci]);
      }
    if (!more) break;
    it = nx;
    x = xn;
  }
}

// the odd last factor of a level: slot `from` of half src -> slot `to` of the other half
template <typename T>
__global__ void k_chain_carry(const JobDev* jobs, int njobs, char* ws, size_t off_T, int src, int from, int to) {
  for (int J = blockIdx.y; J < njobs; J += gridDim.y) {
    const JobDev jb = jobs[J];
    const size_t plane = (size_t)jb.mp * jb.mp;
    T* ub = tplane<T>(ws, off_T, jb.ubuf_off);
    const T* a = ub + (size_t)from * jb.uslot + (size_t)src * 2 * plane;
    T* b = ub + (size_t)to * jb.uslot + (size_t)(1 - src) * 2 * plane;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * plane; i += (size_t)gridDim.x * blockDim.x)
      b[i] = a[i];
  }
}

// K (slot 0 of half `half`) of every block -> interleaved complex128, m x m column-major,
// blocks back to back in job order
template <typename T>
__global__ void k_export_K(const JobDev* jobs, int njobs, char* ws, size_t off_T, int half, double2* out) {
  for (int J = blockIdx.y; J < njobs; J += gridDim.y) {
    const JobDev jb = jobs[J];
    long long off = 0;
    for (int q = 0; q < J; ++q) off += (long long)jobs[q].m * jobs[q].m;
    const size_t plane = (size_t)jb.mp * jb.mp;
    const T* K = tplane<T>(ws, off_T, jb.ubuf_off) + (size_t)half * 2 * plane;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < (long long)jb.m * jb.m;
         idx += (long long)gridDim.x * blockDim.x) {
      const int rr = (int)(idx % jb.m), cc = (int)(idx / jb.m);
      const size_t s = (size_t)rr + (size_t)cc * jb.mp;
      out[off + idx] = make_double2((double)K[s], (double)K[s + plane]);
    }
  }
}

// Gate overlap t = sum_blocks d Tr(Ka^dag Kb) and the weighted squared Frobenius norms
// na = sum_blocks d ||Ka||^2, nb likewise (FP64): per job, kGateParts work-groups sum fixed
// ranges of the entries; k_gate_finish adds the partials in a fixed order and writes
// [F = |t|^2 / (na nb), Re t, Im t, D = sum_blocks d m, na, nb].  For unitaries na = nb = D,
// so F = |t|^2 / D^2; dividing by the norms keeps the drift of FP32 products out of F.
constexpr int kGateParts = 64;
__global__ void __launch_bounds__(256) k_gate_partial(const JobDev* jobs, int njobs, const double2* Ka,
                                                      const double2* Kb, double* part) {
  __shared__ double rr[256], ri[256], ra[256], rb[256];
  for (int J = blockIdx.y; J < njobs; J += gridDim.y) {
    const JobDev jb = jobs[J];
    long long off = 0;
    for (int q = 0; q < J; ++q) off += (long long)jobs[q].m * jobs[q].m;
    const long long n = (long long)jb.m * jb.m;
    const long long per = (n + kGateParts - 1) / kGateParts;
    const long long lo = (long long)blockIdx.x * per, hi = min(n, lo + per);
    double sr = 0.0, si = 0.0, sa = 0.0, sb = 0.0;
    for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const double2 a = Ka[off + i], b = Kb[off + i];
      sr += a.x * b.x + a.y * b.y;  // conj(a) b
      si += a.x * b.y - a.y * b.x;
      sa += a.x * a.x + a.y * a.y;
      sb += b.x * b.x + b.y * b.y;
    }
    rr[threadIdx.x] = sr;
    ri[threadIdx.x] = si;
    ra[threadIdx.x] = sa;
    rb[threadIdx.x] = sb;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) {
        rr[threadIdx.x] += rr[threadIdx.x + h];
        ri[threadIdx.x] += ri[threadIdx.x + h];
        ra[threadIdx.x] += ra[threadIdx.x + h];
        rb[threadIdx.x] += rb[threadIdx.x + h];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      double* pp = part + 4 * ((size_t)J * kGateParts + blockIdx.x);
      pp[0] = rr[0] * jb.d;
      pp[1] = ri[0] * jb.d;
      pp[2] = ra[0] * jb.d;
      pp[3] = rb[0] * jb.d;
    }
    __syncthreads();
  }
}

__global__ void k_gate_finish(const JobDev* jobs, int njobs, const double* part, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double tr = 0.0, ti = 0.0, na = 0.0, nb = 0.0, D = 0.0;
  for (int J = 0; J < njobs; ++J) {
    for (int b = 0; b < kGateParts; ++b) {
      const double* pp = part + 4 * ((size_t)J * kGateParts + b);
      tr += pp[0];
      ti += pp[1];
      na += pp[2];
      nb += pp[3];
    }
    D += (double)jobs[J].d * jobs[J].m;
  }
  out[0] = (tr * tr + ti * ti) / (na * nb);
  out[1] = tr;
  out[2] = ti;
  out[3] = D;
  out[4] = na;
  out[5] = nb;
}

// interleaved complex128 copy of U_j for qoc_propagate
template <typename T>
__global__ void k_export_U(const JobDev* jobs, int njobs, char* ws, size_t off_T, const int* ent_s, const int* ent_q,
                           int r, int seg_j0, int seg_len, double2* out) {
  for (long long e = blockIdx.y; e < (long long)njobs * seg_len; e += gridDim.y) {
  const int J = find_job_by_ent(jobs, njobs, e);
  const JobDev jb = jobs[J];
  const int jl = (int)(e - jb.ent_off);
  if (jl >= job_len(jb, seg_j0, seg_len)) continue;
  const T* U = entry_U<T>(jb, ws, off_T, jl);
  const size_t plane = (size_t)jb.mp * jb.mp;
  double2* dst = out + jb.uout_off + (size_t)(seg_j0 + jl) * jb.m * jb.m;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < (long long)jb.m * jb.m;
       idx += (long long)gridDim.x * blockDim.x) {
    const int rr = (int)(idx % jb.m), cc = (int)(idx / jb.m);
    const size_t s = (size_t)rr + (size_t)cc * jb.mp;
    dst[idx] = make_double2((double)U[s], (double)U[s + plane]);
  }
  }
}

// dst = sum_{i < count} slot[first + i] (fixed order)
template <typename T>
__global__ void k_slot_sum(const JobDev* jobs, int njobs, char* ws, size_t off_T, int dst, int first, int count,
                           int j0) {
  for (int J = blockIdx.y; J < njobs; J += gridDim.y) {
  const JobDev jb = jobs[J];
  if (jb.N - j0 <= 0) continue;
  T* g = tplane<T>(ws, off_T, jb.gbase_off);
  const long long total = 2LL * jb.mp * jb.cc;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    T s = T(0);
    for (int i = 0; i < count; ++i) s += g[(size_t)(first + i) * jb.gslot + idx];
    g[(size_t)dst * jb.gslot + idx] = s;
  }
  }
}

// ===================================================================== profiler
// Opt-in, process-wide launch timing for benchmarks: HIP events from a pre-created
// pool are recorded on the launch stream around each kernel of the hot path.
enum ProfKind {
  PK_GENERATOR = 0, PK_EXPM_GEMM = 1, PK_GATE_CHAIN = 2, PK_SWEEP_FWD = 3, PK_SWEEP_BWD = 4,
  PK_OVERLAP = 5, PK_GRAD_GEMM = 6, PK_GRAD_VECTOR = 7, PK_GRAD_FINISH = 8, PK_OTHER = 9, PK_COUNT = 10
};

struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  size_t dropped = 0;  // launches made while the pool was exhausted (not timed)
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
    if (g_prof.on) ++g_prof.dropped;
    launch();
  }
  QOC_HIP(hipGetLastError());
}

// Norms and (q, s) choice of every slice, without forming the generators (statistics).
__global__ void __launch_bounds__(256) k_slice_norms(const JobDev* jobs, int njobs, const double* u, int Nmax,
                                                     const double* theta, int r, int qmax, int t12, int pow_free,
                                                     int* q_out, int* s_out,
                                                     double* n_out) {
  __shared__ double red[256];
  __shared__ double ujs[kMaxControls + 1];
  const int j = blockIdx.x;
  for (int J = blockIdx.y; J < njobs; J += gridDim.y) {
  const JobDev jb = jobs[J];
  if (j >= jb.N) {
    if (threadIdx.x == 0) {
      q_out[(size_t)J * Nmax + j] = -1;
      s_out[(size_t)J * Nmax + j] = 0;
      n_out[(size_t)J * Nmax + j] = 0.0;
    }
    continue;
  }
  const int m = jb.m, mp = jb.mp, K = jb.K;
  const size_t plane = (size_t)mp * mp;
  __syncthreads();
  if (threadIdx.x <= K) ujs[threadIdx.x] = threadIdx.x == 0 ? 1.0 : u[jb.u_off + (size_t)j * K + threadIdx.x - 1];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double cmax = 0.0;
  for (int c = wave; c < m; c += nw) {
    double cs = 0.0;
    for (int rr = lane; rr < m; rr += 64) {
      const size_t idx = (size_t)rr + (size_t)c * mp;
      double hr = 0.0, hi = 0.0;
      for (int o = 0; o <= K; ++o) {
        hr += ujs[o] * jb.h64[(size_t)(2 * o) * plane + idx];
        hi += ujs[o] * jb.h64[(size_t)(2 * o + 1) * plane + idx];
      }
      cs += hypot(hr, hi);
    }
    cmax = fmax(cmax, warp_sum(cs));
  }
  red[threadIdx.x] = cmax;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nx = jb.dt * red[0];
    int q, s;
    pick_degree(nx, theta, r, qmax, t12, pow_free, &q, &s);
    q_out[(size_t)J * Nmax + j] = q;
    s_out[(size_t)J * Nmax + j] = s;
    n_out[(size_t)J * Nmax + j] = nx;
  }
  __syncthreads();
  }
}

// ===================================================================== host driver
static double fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

static void upload_factorials() {
  static std::mutex mu;
  static std::vector<int> devices_done;
  std::lock_guard<std::mutex> lk(mu);
  int dev = 0;
  QOC_HIP(hipGetDevice(&dev));
  if (std::find(devices_done.begin(), devices_done.end(), dev) != devices_done.end()) return;
  double h[64];
  for (int i = 0; i < 64; ++i) h[i] = 1.0 / fact(i);
  QOC_HIP(hipMemcpyToSymbol(HIP_SYMBOL(kInvFact), h, sizeof(h)));
  QOC_HIP(hipMemcpyToSymbol(HIP_SYMBOL(kT12c), kT12, sizeof(kT12)));
  devices_done.push_back(dev);
}

// ================================================================ GEMM tile variants
// The GEMM kernels are compiled for a few work-group tile shapes per precision; a plan
// uses one (default: the first) and qoc_plan_autotune picks the fastest on the plan's own
// work.  Every shape accumulates each output element over k in the same order, so the
// choice does not change any result bit.
typedef void (*ExpmLaunch)(dim3, hipStream_t, const JobDev*, int, long long, char*, size_t, const int*,
                           const int*, int, int, int, int, int, int, int, int, const int*, int);
typedef void (*PanelLaunch)(dim3, hipStream_t, const JobDev*, const PanelDesc*, int, long long, char*, size_t, int,
                            int);
typedef void (*ChainLaunch)(dim3, hipStream_t, const JobDev*, int, long long, char*, size_t, int, int, int);
struct GemmVariant {
  const char* name;
  int bm, bn;
  ExpmLaunch expm;
  PanelLaunch panel;
  ChainLaunch chain;
  const void* expm_fn;  // for occupancy queries
};
template <typename C>
void launch_expm(dim3 g, hipStream_t st, const JobDev* j, int nj, long long items, char* ws, size_t offT,
                 const int* es, const int* eq, int mode, int step, int r, int j0, int len, int c0, int clen,
                 int skip_n, const int* flags, int gen_b) {
  hipLaunchKernelGGL(k_expm_step<C>, g, dim3(256), 0, st, j, nj, items, ws, offT, es, eq, mode, step, r, j0, len, c0,
                     clen, skip_n, flags, gen_b);
}
template <typename C>
void launch_panel(dim3 g, hipStream_t st, const JobDev* j, const PanelDesc* d, int nd, long long items, char* ws,
                  size_t offT, int vslot, int j0) {
  hipLaunchKernelGGL(k_panel_gemm<C>, g, dim3(256), 0, st, j, d, nd, items, ws, offT, vslot, j0);
}
template <typename C>
void launch_chain(dim3 g, hipStream_t st, const JobDev* j, int nj, long long items, char* ws, size_t offT, int src,
                  int c0, int npairs) {
  hipLaunchKernelGGL(k_chain_step<C>, g, dim3(256), 0, st, j, nj, items, ws, offT, src, c0, npairs);
}
template <typename C>
GemmVariant make_variant(const char* name) {
  return GemmVariant{name, C::BM, C::BN, launch_expm<C>, launch_panel<C>, launch_chain<C>,
                     (const void*)k_expm_step<C>};
}
static const GemmVariant kVariants32[] = {
    make_variant<TileShape<float, 4, 2, 2>>("fp32 128x64"),
    make_variant<TileShape<float, 2, 2, 2>>("fp32 64x64"),
    make_variant<TileShape<float, 2, 4, 2>>("fp32 64x128"),
};
static const GemmVariant kVariants64[] = {
    make_variant<TileShape<double, 2, 2, 2>>("fp64 64x64"),
    make_variant<TileShape<double, 1, 2, 2>>("fp64 32x64"),
    make_variant<TileShape<double, 2, 1, 2>>("fp64 64x32"),
};
constexpr int kNumVariants = 3;
static const GemmVariant& gemm_variant(const qoc_plan_s* P) {
  return P->prec == QOC_C128 ? kVariants64[P->variant] : kVariants32[P->variant];
}

// Tile counts and item offsets of the propagator and panel GEMMs for variant v, the
// persistent grid for its occupancy, and the device copies of both tables (set-up only:
// synchronous copies).
static void apply_variant(qoc_plan_s* P, int v) {
  QOC_REQUIRE(v >= 0 && v < kNumVariants, QOC_ERR_INVALID_ARG, "unknown GEMM variant");
  P->variant = v;
  const GemmVariant& g = gemm_variant(P);
  long long items = 0;
  for (auto& j : P->jobs) {
    j.tiles_m = (j.mp + g.bm - 1) / g.bm;
    j.tiles_n = (j.mp + g.bn - 1) / g.bn;
    j.item_off = items;
    items += (long long)P->echunk * j.tiles_m * j.tiles_n;
  }
  P->expm_items = items;
  long long pitems = 0;
  for (auto& d : P->panels) {
    d.item_off = pitems;
    d.tiles_m = (P->jobs[d.job].mp + g.bm - 1) / g.bm;
    d.tiles_n = (P->jobs[d.job].cc + g.bn - 1) / g.bn;
    pitems += (long long)d.tiles_m * d.tiles_n;
  }
  P->panel_items = pitems;
  int occ = 1;
  QOC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, g.expm_fn, 256, 0));
  P->grid_gemm = std::max(8, P->ncu * std::max(1, occ) / 8 * 8);
  QOC_HIP(hipMemcpy(P->d_jobs.ptr, P->jobs.data(), P->jobs.size() * sizeof(JobDev), hipMemcpyHostToDevice));
  if (!P->panels.empty())
    QOC_HIP(hipMemcpy(P->d_panels.ptr, P->panels.data(), P->panels.size() * sizeof(PanelDesc), hipMemcpyHostToDevice));
}

template <typename T>
struct Driver {
  static int* ent_s(const qoc_plan_s* P, char* ws) { return reinterpret_cast<int*>(ws + P->off_ent); }
  static int* ent_q(const qoc_plan_s* P, char* ws) { return ent_s(P, ws) + P->entries_per_seg; }
  static double* ent_norm(const qoc_plan_s* P, char* ws) {
    return reinterpret_cast<double*>(ws + P->off_ent + (size_t)8 * P->entries_per_seg);
  }
  static size_t sweep_lds(const qoc_plan_s* P) { return P->sweep_lds_elems * sizeof(T); }

  // The workspace copies of the operator products (systems that keep none), at the start of
  // every call that forms propagators: five passes of set-up GEMMs (product_descs).
  static void form_products(qoc_plan_s* P, char* ws, hipStream_t st) {
    if (!P->pw_ws) return;
    typedef typename ProductShape<T>::type Shape;
    const SetupGemmT<T>* d = P->d_pwgemm.as<SetupGemmT<T>>();
    for (int p = 0; p < 5; ++p) {
      const int n = P->pw_pass_begin[p + 1] - P->pw_pass_begin[p];
      const long long items = P->pw_pass_items[p];
      if (n == 0) continue;
      const unsigned grid = (unsigned)std::max<long long>(8, std::min<long long>(P->grid_gemm, (items + 7) / 8 * 8));
      timed(PK_GENERATOR, st, [&] {
        hipLaunchKernelGGL(k_setup_gemm<Shape>, dim3(grid), dim3(256), 0, st, d + P->pw_pass_begin[p], n, items, ws);
      });
    }
  }

  // Propagators of the segment starting at seg_j0.  skip_n > 0 (backward recompute): jobs
  // with N <= skip_n are left alone -- their last segment is this one, whose propagators
  // no later segment overwrote.
  static void expm_segment(qoc_plan_s* P, char* ws, const double* u, int seg_j0, hipStream_t st, int skip_n = 0) {
    const int njobs = (int)P->jobs.size();
    const JobDev* dj = P->d_jobs.as<JobDev>();
    int* flags = reinterpret_cast<int*>(ws + P->off_flags);
    const int L = P->seg_len;
    const dim3 grid(P->grid_gemm);
    // the segment in chunks of echunk slices: Taylor scratch for one chunk, U of every
    // slice kept
    for (int c0 = 0; c0 < L; c0 += P->echunk) {
      const int clen = std::min(P->echunk, L - c0);
      const int groups = (clen + GEN_SG - 1) / GEN_SG;
      // too few (job, slice group) work-groups to keep every CU busy with several (and to
      // even out blocks of different sizes), each reading large operator planes: split each
      // over column ranges
      const long long wgs = (long long)njobs * groups, target = 16LL * P->ncu;
      const int csplit = P->gen_split > 0 ? std::min(P->gen_split, std::max(1, P->max_mp / 16))
                         : wgs >= target || P->max_mp < 64
                             ? 1
                             : (int)std::min<long long>((target + wgs - 1) / wgs, std::max(1, P->max_mp / 16));
      if (csplit == 1) {
        timed(PK_GENERATOR, st, [&] {
          hipLaunchKernelGGL(k_generator<T>, dim3(njobs * groups), dim3(256), 0, st, dj, njobs, u, seg_j0, L, c0,
                             clen, groups, ws, P->off_T, ent_s(P, ws), ent_q(P, ws), ent_norm(P, ws), flags,
                             P->d_theta.as<double>(), P->r, P->qmax, P->t12, P->pow_free, P->smax, P->norm_bound,
                             skip_n);
        });
      } else {
        timed(PK_GENERATOR, st, [&] {
          // the chunk's entries of ent_norm collect maxima: zero them first
          hipLaunchKernelGGL(k_gen_zero, dim3((clen + 255) / 256, (unsigned)std::min(njobs, 65535)), dim3(256), 0, st,
                             dj, njobs, c0, clen, ent_norm(P, ws));
          hipLaunchKernelGGL(k_gen_norms, dim3((unsigned)(wgs * csplit)), dim3(256), 0, st, dj, njobs, u, seg_j0, L,
                             c0, clen, groups, csplit, ent_norm(P, ws), skip_n);
          hipLaunchKernelGGL(k_gen_pick, dim3((unsigned)wgs), dim3(64), 0, st, dj, njobs, u, seg_j0, L, c0, clen,
                             groups, ent_s(P, ws), ent_q(P, ws), ent_norm(P, ws), flags, P->d_theta.as<double>(),
                             P->r, P->qmax, P->t12, P->pow_free, P->smax, P->norm_bound, skip_n);
          hipLaunchKernelGGL(k_gen_form<T>, dim3((unsigned)(wgs * csplit)), dim3(256), 0, st, dj, njobs, u, seg_j0,
                             L, c0, clen, groups, csplit, ws, P->off_T, ent_s(P, ws), ent_q(P, ws), P->r, P->pow_free,
                             skip_n);
        });
      }
      auto step = [&](int mode, int s) {
        timed(PK_EXPM_GEMM, st, [&] {
          gemm_variant(P).expm(grid, st, dj, njobs, P->expm_items, ws, P->off_T, ent_s(P, ws), ent_q(P, ws), mode, s,
                               P->r, seg_j0, L, c0, clen, skip_n, flags, P->pow_free && P->r == 3 ? 1 : 0);
        });
      };
      // powers Y^2 .. Y^r (those the generator formed are skipped)
      for (int i = 2 + P->pow_free; i <= P->r; ++i) step(STEP_POWER, i);
      if (P->t12) {
        step(STEP_T12, 1);
        step(STEP_T12, 2);
      }
      for (int t = 1; t <= P->qmax - 1; ++t) step(STEP_HORNER, t);
      for (int t = 1; t <= P->smax; ++t) step(STEP_SQUARE, t);
    }
  }

  static void sweep(qoc_plan_s* P, char* ws, int dir, int seg_j0, hipStream_t st) {
    const int njobs = (int)P->jobs.size();
    const JobDev* dj = P->d_jobs.as<JobDev>();
    if (P->coop) {
      int* ctl = reinterpret_cast<int*>(ws + P->off_sync) + (size_t)dir * 4 * njobs;
      int* flags = reinterpret_cast<int*>(ws + P->off_flags);
      const dim3 grid(P->coop_w, njobs);
      // one group per job: 4 columns per wave, at least the 128 threads of the reduction
      const int threads = P->coop_w == 1 ? std::min(1024, std::max(256, 16 * P->max_mp)) : 1024;
      timed(dir == 0 ? PK_SWEEP_FWD : PK_SWEEP_BWD, st, [&] {
        unsigned long long* xg = reinterpret_cast<unsigned long long*>(ws + P->off_xchg) + (size_t)dir * P->xchg_words;
        const int nz = (int)(2 * P->xchg_words);
        hipLaunchKernelGGL(k_zero_ints, dim3((4 * njobs + 255) / 256), dim3(256), 0, st, ctl, 4 * njobs);
        hipLaunchKernelGGL(k_zero_ints, dim3((nz + 255) / 256), dim3(256), 0, st, reinterpret_cast<int*>(xg), nz);
        const int mode = (P->sweep_mode & QOC_SWEEP_SOLO ? 1 : 0) |
                         (P->sweep_mode & (dir == 0 ? QOC_SWEEP_TEST_STALL_FWD : QOC_SWEEP_TEST_STALL_BWD) ? 2 : 0);
        if (dir == 0)
          hipLaunchKernelGGL((k_sweep_coop<T, 0>), grid, dim3(threads), P->coop_lds, st, dj, njobs, ws, P->off_T,
                             ent_s(P, ws), ent_q(P, ws), P->r, seg_j0, P->seg_len, ctl, flags, xg, mode);
        else
          hipLaunchKernelGGL((k_sweep_coop<T, 1>), grid, dim3(threads), P->coop_lds, st, dj, njobs, ws, P->off_T,
                             ent_s(P, ws), ent_q(P, ws), P->r, seg_j0, P->seg_len, ctl, flags, xg, mode);
      });
      return;
    }
    if (dir == 0)
      timed(PK_SWEEP_FWD, st, [&] {
        hipLaunchKernelGGL((k_sweep<T, 0>), dim3(njobs), dim3(1024), sweep_lds(P), st, dj, njobs, ws, P->off_T,
                           ent_s(P, ws), ent_q(P, ws), P->r, seg_j0, P->seg_len);
      });
    else
      timed(PK_SWEEP_BWD, st, [&] {
        hipLaunchKernelGGL((k_sweep<T, 1>), dim3(njobs), dim3(1024), sweep_lds(P), st, dj, njobs, ws, P->off_T,
                           ent_s(P, ws), ent_q(P, ws), P->r, seg_j0, P->seg_len);
      });
  }

  // Timing pass of the autotuner: the first segment's propagators and one panel GEMM.
  static void tune_pass(qoc_plan_s* P, const double* u, char* ws, hipStream_t st) {
    int* flags = reinterpret_cast<int*>(ws + P->off_flags);
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, flags, 16);
    form_products(P, ws, st);
    expm_segment(P, ws, u, 0, st);
    gemm_variant(P).panel(dim3(P->grid_gemm), st, P->d_jobs.as<JobDev>(), P->d_panels.as<PanelDesc>(),
                          (int)P->panels.size(), P->panel_items, ws, P->off_T, P->Kmax + 1, 0);
  }

  // K of every block: propagators of the (single) segment, then the product tree.
  static void gate(qoc_plan_s* P, const double* u, double2* out, char* ws, hipStream_t st) {
    const int njobs = (int)P->jobs.size();
    const JobDev* dj = P->d_jobs.as<JobDev>();
    int* flags = reinterpret_cast<int*>(ws + P->off_flags);
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, flags, 16);
    form_products(P, ws, st);
    expm_segment(P, ws, u, 0, st);
    int cnt = P->Nmax, src = 0;
    while (cnt > 1) {
      const int npairs = cnt / 2;
      for (int c0 = 0; c0 < npairs; c0 += P->echunk)
        timed(PK_GATE_CHAIN, st, [&] {
          gemm_variant(P).chain(dim3(P->grid_gemm), st, dj, njobs, P->expm_items, ws, P->off_T, src, c0, npairs);
        });
      if (cnt & 1)
        timed(PK_OTHER, st, [&] {
          hipLaunchKernelGGL(k_chain_carry<T>, dim3(64, (unsigned)njobs), dim3(256), 0, st, dj, njobs, ws, P->off_T,
                             src, cnt - 1, npairs);
        });
      cnt = (cnt + 1) / 2;
      src = 1 - src;
    }
    timed(PK_OTHER, st, [&] {
      hipLaunchKernelGGL(k_export_K<T>, dim3(64, (unsigned)njobs), dim3(256), 0, st, dj, njobs, ws, P->off_T, src,
                         out);
    });
  }

  static void propagate(qoc_plan_s* P, const double* u, double2* out, char* ws, hipStream_t st) {
    const int njobs = (int)P->jobs.size();
    int* flags = reinterpret_cast<int*>(ws + P->off_flags);
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, flags, 16);
    form_products(P, ws, st);
    for (int sg = 0; sg < P->nseg; ++sg) {
      const int j0 = sg * P->seg_len;
      expm_segment(P, ws, u, j0, st);
      timed(PK_OTHER, st, [&] {
        hipLaunchKernelGGL(k_export_U<T>, dim3(16, (unsigned)std::min<long long>(P->entries_per_seg, 32768)), dim3(256), 0, st,
                           P->d_jobs.as<JobDev>(), njobs, ws, P->off_T, ent_s(P, ws), ent_q(P, ws), P->r, j0,
                           P->seg_len, out);
      });
    }
  }

  static void run(qoc_plan_s* P, const double* u, const void* psi0, const void* psif, double* out, double* grad,
                  char* ws, hipStream_t st) {
    const int njobs = (int)P->jobs.size();
    const JobDev* dj = P->d_jobs.as<JobDev>();
    const ProbDev* dpr = P->d_probs.as<ProbDev>();
    int* flags = reinterpret_cast<int*>(ws + P->off_flags);
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, flags, 16);  // status ints only
    form_products(P, ws, st);
    timed(PK_OTHER, st, [&] {
      hipLaunchKernelGGL(k_states_in<T>, dim3(std::max(1, std::min(64, 8192 / njobs)), std::min(njobs, 32768)), dim3(256), 0, st, dj, njobs, (const double2*)psi0,
                         (const double2*)psif, ws, P->off_T, flags);
    });
    auto objective = [&](hipStream_t s) {
      timed(PK_OVERLAP, s, [&] {
        hipLaunchKernelGGL(k_overlap<T>, dim3(P->P), dim3(1024), 0, s, dj, dpr, ws, P->off_T, flags, out);
      });
    };
    if (P->nseg == 1 && P->coop_serial) {
      // every propagator stays resident, but the two co-operative sweeps do not fit on the
      // CUs together: one after the other
      expm_segment(P, ws, u, 0, st);
      sweep(P, ws, 0, 0, st);
      objective(st);
      sweep(P, ws, 1, 0, st);
      hipLaunchKernelGGL(k_fold_flags, dim3(1), dim3(64), 0, st, flags, P->P, out);
    } else if (P->nseg == 1) {
      // every propagator stays resident: the two sweeps are independent and run side by
      // side, the backward one on the plan's second stream (fork/join by events)
      expm_segment(P, ws, u, 0, st);
      QOC_HIP(hipEventRecord(P->ev_fork, st));
      QOC_HIP(hipStreamWaitEvent(P->st2, P->ev_fork, 0));
      sweep(P, ws, 1, 0, P->st2);
      QOC_HIP(hipEventRecord(P->ev_join, P->st2));
      sweep(P, ws, 0, 0, st);
      objective(st);
      QOC_HIP(hipStreamWaitEvent(st, P->ev_join, 0));
      // status bits raised by the backward sweep after the objective was written
      hipLaunchKernelGGL(k_fold_flags, dim3(1), dim3(64), 0, st, flags, P->P, out);
    } else {
      // forward: propagators of a segment, then the sequential sweep through it
      for (int sg = 0; sg < P->nseg; ++sg) {
        expm_segment(P, ws, u, sg * P->seg_len, st);
        sweep(P, ws, 0, sg * P->seg_len, st);
      }
      objective(st);
      // backward: the last segment's propagators are resident; earlier ones are recomputed
      for (int sg = P->nseg - 1; sg >= 0; --sg) {
        if (sg != P->nseg - 1) expm_segment(P, ws, u, sg * P->seg_len, st, (sg + 1) * P->seg_len);
        sweep(P, ws, 1, sg * P->seg_len, st);
      }
      // status bits raised by the backward sweeps and recomputed slices after the objective
      // was written
      hipLaunchKernelGGL(k_fold_flags, dim3(1), dim3(64), 0, st, flags, P->P, out);
    }
    gradient(P, u, out, grad, ws, st);
  }

  // Objective only: propagators and the forward sweep, segment by segment (nothing is
  // recomputed: each segment's propagators are used once), then the overlap.
  static void objective_only(qoc_plan_s* P, const double* u, const void* psi0, const void* psif, double* out,
                             char* ws, hipStream_t st) {
    const int njobs = (int)P->jobs.size();
    const JobDev* dj = P->d_jobs.as<JobDev>();
    const ProbDev* dpr = P->d_probs.as<ProbDev>();
    int* flags = reinterpret_cast<int*>(ws + P->off_flags);
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, flags, 16);
    form_products(P, ws, st);
    timed(PK_OTHER, st, [&] {
      hipLaunchKernelGGL(k_states_in<T>, dim3(std::max(1, std::min(64, 8192 / njobs)), std::min(njobs, 32768)),
                         dim3(256), 0, st, dj, njobs, (const double2*)psi0, (const double2*)psif, ws, P->off_T, flags);
    });
    for (int sg = 0; sg < P->nseg; ++sg) {
      expm_segment(P, ws, u, sg * P->seg_len, st);
      sweep(P, ws, 0, sg * P->seg_len, st);
    }
    timed(PK_OVERLAP, st, [&] {
      hipLaunchKernelGGL(k_overlap<T>, dim3(P->P), dim3(1024), 0, st, dj, dpr, ws, P->off_T, flags, out);
    });
  }

  // Exact gradient by the Frechet series over R sub-steps (see the file header).
  static void gradient(qoc_plan_s* P, const double* u, double* out, double* grad, char* ws, hipStream_t st) {
    const int njobs = (int)P->jobs.size();
    const JobDev* dj = P->d_jobs.as<JobDev>();
    const ProbDev* dpr = P->d_probs.as<ProbDev>();
    const int R = P->R, Q = P->Q, K = P->Kmax;
    const int slotA0 = K + 1, slotA1 = K + 2, slotS = K + 3, bank0 = K + 4;
    // per-job vector kernels: about 8k work-groups in total, at most 256 per job
    const dim3 eg(std::max(1, std::min(256, 8192 / njobs)), std::min(njobs, 32768));
    const PanelDesc* dp = P->d_panels.as<PanelDesc>();
    const int npanel = (int)P->panels.size();
    const int C = P->chunk;
    if (P->small_grad && njobs <= 65535) {
      const size_t hbytes = (size_t)(K + 1) * 2 * P->max_mp * P->max_mp * sizeof(T);
      const int hstage = hbytes <= 32768 ? 1 : 0;
      const size_t lds = (size_t)R * Q * kSmallGradRows * 2 * sizeof(double) + (hstage ? hbytes : 0);
      for (int j0 = 0; j0 < P->Nmax; j0 += C) {
        timed(PK_GRAD_VECTOR, st, [&] {
          hipLaunchKernelGGL(k_grad_small<T>, dim3((unsigned)P->max_cc, (unsigned)njobs), dim3(kSmallGradRows), lds, st,
                             dj, njobs, ws, P->off_T, P->off_gacc, u, P->d_w.as<double>(), R, Q, j0, C, hstage);
        });
        timed(PK_GRAD_FINISH, st, [&] {
          hipLaunchKernelGGL(k_grad_finish, dim3((C * K + 255) / 256, P->P), dim3(256), 0, st, dj, dpr, ws,
                             P->off_gacc, j0, C, R, out, grad);
        });
      }
      return;
    }
    for (int j0 = 0; j0 < P->Nmax; j0 += C) {
      auto gemm = [&](int vslot) {
        timed(PK_GRAD_GEMM, st, [&] {
          gemm_variant(P).panel(dim3(P->grid_gemm), st, dj, dp, npanel, P->panel_items, ws, P->off_T, vslot, j0);
        });
      };
      auto combine = [&](double sign_over, int out_slot, int acc_slot) {
        timed(PK_GRAD_VECTOR, st, [&] {
          hipLaunchKernelGGL(k_series_combine<T>, eg, dim3(256), 0, st, dj, njobs, ws, P->off_T, u, j0, C, sign_over,
                             R, out_slot, acc_slot);
        });
      };
      auto slot_sum = [&](int dst, int first, int count) {
        timed(PK_GRAD_VECTOR, st, [&] {
          hipLaunchKernelGGL(k_slot_sum<T>, eg, dim3(256), 0, st, dj, njobs, ws, P->off_T, dst, first, count, j0);
        });
      };
      // b-series, r = R-1 .. 0:  b_0 = lambda^{(r)}, b_{i+1} = +i (dt/R) H_j b_i / (i+1);
      // lambda^{(r-1)} = exp(-Y) lambda^{(r)} = sum_i b_i
      timed(PK_GRAD_VECTOR, st, [&] {
        hipLaunchKernelGGL(k_chunk_load<T>, eg, dim3(256), 0, st, dj, njobs, ws, P->off_T, 1, bank0 + (R - 1) * Q, j0,
                           C);
      });
      for (int rr = R - 1; rr >= 0; --rr) {
        const int bank = bank0 + rr * Q;
        for (int i = 0; i + 1 < Q; ++i) {
          gemm(bank + i);
          combine(1.0 / (i + 1), bank + i + 1, -1);
        }
        if (rr > 0) slot_sum(bank - Q, bank, Q);
      }
      // a-series, r = 0 .. R-1: a_0 = psi^{(r)}, a_{t+1} = -i (dt/R) H_j a_t / (t+1);
      // the dot products take every (i, t) with i + t <= Q - 1
      timed(PK_GRAD_VECTOR, st, [&] {
        hipLaunchKernelGGL(k_chunk_load<T>, eg, dim3(256), 0, st, dj, njobs, ws, P->off_T, 0, slotA0, j0, C);
      });
      int cur = slotA0, nxt = slotA1;
      bool first_dot = true;
      for (int rr = 0; rr < R; ++rr) {
        const int bank = bank0 + rr * Q;
        const bool need_next_state = rr + 1 < R;
        if (need_next_state) slot_sum(slotS, cur, 1);
        for (int t = 0; t < Q; ++t) {
          gemm(cur);
          const double* wt = P->d_w.as<double>() + (size_t)t * Q;
          timed(PK_GRAD_VECTOR, st, [&] {
            const dim3 dg(std::max(1, std::min((P->max_cc + 3) / 4, 8192 / njobs)), std::min(njobs, 32768));
            if (P->Kmax <= 2)
              hipLaunchKernelGGL((k_series_dot<T, 2>), dg, dim3(256), 0, st, dj, njobs, ws, P->off_T, P->off_gacc,
                                 bank, Q - t, wt, first_dot ? 1 : 0, j0);
            else
              hipLaunchKernelGGL((k_series_dot<T, 8>), dg, dim3(256), 0, st, dj, njobs, ws, P->off_T, P->off_gacc,
                                 bank, Q - t, wt, first_dot ? 1 : 0, j0);
          });
          first_dot = false;
          if (t + 1 < Q || need_next_state) {
            combine(-1.0 / (t + 1), nxt, need_next_state ? slotS : -1);
            std::swap(cur, nxt);
          }
        }
        // a_0 of the next sub-step is psi^{(r+1)} = sum_t a_t, held in slotS
        if (need_next_state) slot_sum(cur, slotS, 1);
      }
      timed(PK_GRAD_FINISH, st, [&] {
        hipLaunchKernelGGL(k_grad_finish, dim3((C * K + 255) / 256, P->P), dim3(256), 0, st, dj, dpr, ws, P->off_gacc,
                           j0, C, R, out, grad);
      });
    }
  }
};

// ------------------------------------------------------------------- plan construction
struct ProblemSpec {
  qoc_system_s* sys;
  int N;
  double dt;
  // the blocks this problem carries (all of the system's, or a chosen subset); state_off
  // is the block's offset in this problem's panel
  std::vector<qoc_system_s::Block> blocks;
};

static ProblemSpec all_blocks(qoc_system_s* sys, int N, double dt) {
  QOC_REQUIRE(sys, QOC_ERR_INVALID_ARG, "null system");
  return ProblemSpec{sys, N, dt, sys->blocks};
}

// The operator products of qoc_system_s::pw64 / pw32 (see there), formed once per system
// on the FP64 matrix cores (product_descs' five passes over all blocks) and kept in the
// precision a plan asks for (FP64 for complex128 plans, FP32 for complex64 ones).
static void ensure_powers(qoc_system_s* S, bool f64) {
  if (S->K > kMaxPowK || (f64 ? S->pw64.ptr : S->pw32.ptr) != nullptr) return;
  const int K = S->K, npw = pair_count(K) + triple_count(K);
  int64_t elems = 0;
  S->pw_off.clear();
  for (auto& b : S->blocks) {
    S->pw_off.push_back(elems);
    elems += (int64_t)npw * 2 * b.mp * b.mp;
  }
  DeviceBuffer prod((size_t)elems * sizeof(double));
  hipStream_t st = nullptr;
  typedef TileShape<double, 2, 2, 2> Shape;
  std::vector<SetupGemmT<double>> pass[5];
  long long items[5] = {0, 0, 0, 0, 0};
  for (size_t bi = 0; bi < S->blocks.size(); ++bi) {
    const auto& blk = S->blocks[bi];
    product_descs<double>(S->h64.as<double>() + blk.h_off, 0, prod.as<double>() + S->pw_off[bi], 0, K, blk.mp,
                          Shape::BM, Shape::BN, pass, items);
  }
  for (int p = 0; p < 5; ++p) {
    if (pass[p].empty()) continue;
    DeviceBuffer dd(pass[p].size() * sizeof(SetupGemmT<double>));
    QOC_HIP(hipMemcpy(dd.ptr, pass[p].data(), pass[p].size() * sizeof(SetupGemmT<double>), hipMemcpyHostToDevice));
    const int grid = (int)std::min<long long>(2048, (items[p] + 7) / 8 * 8);
    hipLaunchKernelGGL(k_setup_gemm<Shape>, dim3(std::max(8, grid)), dim3(256), 0, st, dd.as<SetupGemmT<double>>(),
                       (int)pass[p].size(), items[p], nullptr);
    QOC_HIP(hipGetLastError());
    QOC_HIP(hipStreamSynchronize(st));
  }
  if (f64) {
    S->pw64 = std::move(prod);
  } else {
    S->pw32.alloc((size_t)elems * sizeof(float));
    hipLaunchKernelGGL(k_planes_to_float, dim3(4096), dim3(256), 0, st, prod.as<double>(), S->pw32.as<float>(),
                       (size_t)elems);
    QOC_HIP(hipGetLastError());
    QOC_HIP(hipStreamSynchronize(st));
  }
}

// How a plan's generator gets Y^2 and Y^3: 0 by power products (some system has more than
// kMaxPowK controls); 1 from operator products kept with every system; 2 from products formed
// at the start of every call in the workspace for the systems that keep none.  The products
// still missing are formed and kept with their systems when they fit an eighth of the free
// device memory: a large batch of distinct Hamiltonians (the 256-ring batch: 97 GB of
// products) keeps that memory for its propagators and forms each problem group's products
// per call instead (a few per cent of the call's products).  Call it before the workspace
// budget is read from the free memory.
static std::atomic<int> g_products_policy{0};  // qoc_set_products_policy
static int prepare_powers(const std::vector<ProblemSpec>& probs, bool f64) {
  for (auto& pr : probs)
    if (pr.sys->K > kMaxPowK) return 0;
  std::vector<qoc_system_s*> missing;
  size_t bytes = 0;
  for (auto& pr : probs) {
    qoc_system_s* S = pr.sys;
    if ((f64 ? S->pw64.ptr : S->pw32.ptr) != nullptr ||
        std::find(missing.begin(), missing.end(), S) != missing.end())
      continue;
    missing.push_back(S);
    size_t planes = 0;
    for (auto& b : S->blocks) planes += (size_t)b.mp * b.mp;
    bytes += (size_t)(pair_count(S->K) + triple_count(S->K)) * 2 * planes * (f64 ? sizeof(double) : sizeof(float));
  }
  if (missing.empty()) return 1;
  size_t free_b = 0, total_b = 0;
  QOC_HIP(hipMemGetInfo(&free_b, &total_b));
  if (g_products_policy.load() == 0 && bytes <= free_b / 8) {
    for (auto* S : missing) ensure_powers(S, f64);
    return 1;
  }
  return 2;
}

// whether system S keeps operator products in the plan's precision
static bool keeps_products(const qoc_system_s* S, bool f64) {
  return (f64 ? S->pw64.ptr : S->pw32.ptr) != nullptr;
}

// Default workspace budget: 85 % of the free device memory (the rest for the caller's
// tensors and the allocator), at most 240 GiB of the 288 GB part.
static size_t default_budget() {
  size_t free_b = 0, total_b = 0;
  QOC_HIP(hipMemGetInfo(&free_b, &total_b));
  return std::min<size_t>((size_t)240 << 30, free_b / 20 * 17);
}

// Device descriptors of the workspace products (Driver::form_products): every (system,
// block) key's five passes, the passes concatenated.  The products' addresses are workspace
// byte offsets (off_T + element offset); the operators are the systems' own planes.
template <typename T>
static void upload_product_descs(qoc_plan_s* P, const std::vector<std::pair<const qoc_system_s*, int>>& keys,
                                 const std::vector<long long>& off) {
  typedef typename ProductShape<T>::type Shape;
  std::vector<SetupGemmT<T>> pass[5];
  long long items[5] = {0, 0, 0, 0, 0};
  for (size_t k = 0; k < keys.size(); ++k) {
    const qoc_system_s* S = keys[k].first;
    const auto& b = S->blocks[keys[k].second];
    const T* H = std::is_same<T, double>::value ? reinterpret_cast<const T*>(S->h64.as<double>() + b.h_off)
                                                : reinterpret_cast<const T*>(S->h32.as<float>() + b.h_off);
    T* PW = reinterpret_cast<T*>((uintptr_t)(P->off_T + (size_t)off[k] * sizeof(T)));
    product_descs<T>(H, 0, PW, 1, S->K, b.mp, Shape::BM, Shape::BN, pass, items);
  }
  std::vector<SetupGemmT<T>> all;
  for (int p = 0; p < 5; ++p) {
    P->pw_pass_begin[p] = (int)all.size();
    P->pw_pass_items[p] = items[p];
    all.insert(all.end(), pass[p].begin(), pass[p].end());
  }
  P->pw_pass_begin[5] = (int)all.size();
  P->d_pwgemm.alloc(all.size() * sizeof(SetupGemmT<T>));
  QOC_HIP(hipMemcpy(P->d_pwgemm.ptr, all.data(), all.size() * sizeof(SetupGemmT<T>), hipMemcpyHostToDevice));
}

// pow_mode: -1 decides how the generator gets its powers (prepare_powers); 0 / 1 / 2 take a
// decision made for the whole batch.  parent (a problem group's plan): the batch plan whose
// numerical choices the group takes over -- products, Frechet sub-steps and terms, gradient
// route -- so that grouping changes no result.
static qoc_plan_s* build_plan(const std::vector<ProblemSpec>& probs, int precision, double u_bound, size_t max_ws,
                              int pow_mode = -1, const qoc_plan_s* parent = nullptr) {
  QOC_REQUIRE(precision == QOC_C128 || precision == QOC_C64, QOC_ERR_INVALID_ARG, "unknown precision");
  QOC_REQUIRE(std::isfinite(u_bound) && u_bound >= 0.0, QOC_ERR_INVALID_ARG, "u_bound must be finite and >= 0");
  QOC_REQUIRE(!probs.empty(), QOC_ERR_INVALID_ARG, "no problems");
  for (auto& pr : probs) {
    QOC_REQUIRE(pr.sys, QOC_ERR_INVALID_ARG, "null system");
    QOC_REQUIRE(pr.N >= 1 && pr.N <= (1 << 24), QOC_ERR_INVALID_ARG, "N must be in 1..2^24");
    QOC_REQUIRE(std::isfinite(pr.dt) && pr.dt > 0.0, QOC_ERR_INVALID_ARG, "dt must be positive and finite");
  }
  upload_factorials();
  auto P = std::make_unique<qoc_plan_s>();
  P->P = (int)probs.size();
  P->prec = precision;
  P->u_bound = u_bound;
  const bool f64 = precision == QOC_C128;
  P->elem = f64 ? 8 : 4;
  const double* theta = f64 ? kTaylorTheta64 : kTaylorTheta32;
  P->r = f64 ? 4 : 3;
  P->qmax = f64 ? 6 : 4;  // degrees up to 24 (FP64) / 12 (FP32)
  P->t12 = f64 ? 0 : 1;
  // Y^2 and Y^3 from the operator products when every system has them (few controls)
  const int pmode = parent ? parent->pw_mode : (pow_mode < 0 ? prepare_powers(probs, f64) : pow_mode);
  P->pw_mode = pmode;
  P->pow_free = pmode > 0 ? 2 : 0;
  const double unit = f64 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
  double nb = 0.0;
  int max_mp = 0;
  for (auto& pr : probs) {
    P->Nmax = std::max(P->Nmax, pr.N);
    P->Kmax = std::max(P->Kmax, pr.sys->K);
    // norm bound by the triangle inequality on the exact block 1-norms
    for (auto& b : pr.blocks) {
      double v = b.norm1[0];
      for (int k = 1; k <= pr.sys->K; ++k) v += u_bound * b.norm1[k];
      nb = std::max(nb, pr.dt * v);
      max_mp = std::max(max_mp, b.mp);
    }
    if (std::find(P->systems.begin(), P->systems.end(), pr.sys) == P->systems.end()) P->systems.push_back(pr.sys);
  }
  P->norm_bound = nb;
  {
    // squarings the per-slice choice can pick for any norm in (0, nb]: the choice is
    // piecewise constant between the points theta_{qr} 2^s, so evaluate just above each
    auto choose_s = [&](double nx) {
      int q = 0, sq = 0;
      pick_degree(nx, theta, P->r, P->qmax, P->t12, P->pow_free, &q, &sq);
      return sq;
    };
    int smax = choose_s(nb);
    std::vector<int> degrees;
    for (int q = 1; q <= P->qmax; ++q) degrees.push_back(q * P->r);
    degrees.push_back(12);
    for (int p : degrees)
      for (int sq = 0; sq < 62; ++sq) {
        const double x = std::ldexp(theta[p], sq);
        if (x >= nb) break;
        smax = std::max(smax, choose_s(std::nextafter(x, 1e300)));
      }
    P->smax = smax;
  }
  QOC_REQUIRE(P->smax <= 40, QOC_ERR_NUMERIC, "dt * ||H|| bound too large");
  {
    // Frechet series: R sub-steps and Q terms, the cheapest R*Q with theta^Q/Q! <= unit/8
    // for theta = nb/R, keeping theta <= 3.5 so that the alternating terms (largest
    // ~e^theta) lose at most a factor ~33 to cancellation
    auto terms_for = [&](double th) {
      int Q = 2;
      while (Q < 80 && std::pow(th, Q) / fact(Q) > unit / 8) ++Q;
      return Q;
    };
    int bestR = 1, bestQ = 0;
    long best = -1;
    for (int R = 1; R <= 1 << 20; R *= 2) {
      const double th = nb / R;
      if (th > 3.5) continue;
      const int Q = terms_for(th);
      if (best < 0 || (long)R * Q < best) { best = (long)R * Q; bestR = R; bestQ = Q; }
      if (th < 0.5) break;
    }
    QOC_REQUIRE(bestQ > 0, QOC_ERR_NUMERIC, "dt * ||H|| bound too large for the gradient series");
    P->R = bestR;
    P->Q = bestQ;
  }
  P->small_grad = max_mp <= kSmallGradMaxWidth && P->R * P->Q <= kSmallGradMaxRQ;
  if (parent) {  // the parent's bound covers this subset: its choices hold here too
    P->R = parent->R;
    P->Q = parent->Q;
    P->small_grad = parent->small_grad;
  }
  QOC_REQUIRE(max_mp <= 4096, QOC_ERR_UNSUPPORTED, "blocks larger than 4096 are not supported by the sweep kernels");
  P->max_mp = max_mp;
  size_t lds_elems = 0;
  for (auto& pr : probs)
    for (auto& b : pr.blocks) {
      // copies: the dimension of a ring group's irrep (1 or 2; one for S_n blocks)
      QOC_REQUIRE(b.d == 1 || b.d == 2, QOC_ERR_UNSUPPORTED, "blocks with more than two copies");
      lds_elems = std::max(lds_elems, (size_t)2 * b.d * b.mp * (1 + sweep_kgroups(b.mp, (int)P->elem)));
    }
  P->sweep_lds_elems = lds_elems;
  QOC_REQUIRE(lds_elems * P->elem <= 160 * 1024, QOC_ERR_UNSUPPORTED, "block panel too large for the LDS-resident sweep");
  const int K = P->Kmax;
  const int nslots = K + 4 + P->R * P->Q;
  P->nslots = nslots;
  // per-slice bytes: U kept for the segment (uplanes planes: U alone, or U and room for
  // the gate product tree), Taylor scratch (Y..Y^r, two ping-pong buffers) for one chunk;
  // fixed state bytes
  size_t per_plane = 0, per_scratch = 0, fixed = 0;
  for (auto& pr : probs)
    for (auto& b : pr.blocks) {
      per_plane += (size_t)b.mp * b.mp * P->elem;
      per_scratch += (size_t)(P->r + 2) * 2 * b.mp * b.mp * P->elem;
      fixed += (size_t)2 * b.mp * ((size_t)(pr.N + 1) * b.d + (size_t)pr.N * b.d) * P->elem;
    }
  // operator products held in the workspace: one copy per (system, block) whose system keeps
  // none, in first-use order
  std::vector<std::pair<const qoc_system_s*, int>> pw_keys;
  if (P->pow_free)
    for (auto& pr : probs) {
      if (keeps_products(pr.sys, f64)) continue;
      const int npw = pair_count(pr.sys->K) + triple_count(pr.sys->K);
      for (auto& b : pr.blocks) {
        const std::pair<const qoc_system_s*, int> key{pr.sys, b.index};
        if (std::find(pw_keys.begin(), pw_keys.end(), key) != pw_keys.end()) continue;
        pw_keys.push_back(key);
        fixed += (size_t)npw * 2 * b.mp * b.mp * P->elem;
      }
    }
  P->pw_ws = !pw_keys.empty();
  std::vector<long long> pw_key_off(pw_keys.size(), -1);
  const size_t budget = max_ws ? max_ws : default_budget();
  // The segment length, Taylor chunk and gradient chunk for uplanes planes per slice; true
  // when every propagator is resident (one segment).
  auto plan_memory = [&](int uplanes) {
    const size_t per_slice = (size_t)uplanes * per_plane;
    int chunk = std::min(P->Nmax, 2048);
    auto grad_bytes = [&](int ch) {
      size_t g = 0;
      for (auto& pr : probs)
        for (auto& b : pr.blocks) {
          const int cc = (ch * b.d + 15) / 16 * 16;
          g += (size_t)nslots * 2 * b.mp * cc * P->elem + (size_t)cc * K * 16;
        }
      return g;
    };
    while (chunk > 16 && fixed + grad_bytes(chunk) + per_slice + per_scratch > budget) chunk /= 2;
    // A smaller gradient chunk (down to 16 slices: more, narrower gradient launches, the same
    // work) is preferred when it lets every propagator stay resident (no recompute in the
    // backward sweep).  When the propagators must be segmented anyway, the gradient slots
    // take at most an eighth of the budget, so that the segments stay long: each segment
    // costs a round of launches and every segment but the last is formed twice.
    const long long ec_min = std::min(P->Nmax, 8);
    auto resident = [&](int ch) {
      return fixed + grad_bytes(ch) + (size_t)P->Nmax * per_slice + (size_t)ec_min * per_scratch <= budget;
    };
    if (!resident(chunk)) {
      int ch = chunk;
      while (ch > 16 && !resident(ch)) ch /= 2;
      if (resident(ch)) {
        chunk = ch;
      } else {
        while (chunk > 16 && grad_bytes(chunk) > budget / 8) chunk /= 2;
      }
    }
    P->chunk = chunk;
    const size_t need = fixed + grad_bytes(chunk);
    const size_t avail = budget > need ? budget - need : 0;
    if ((size_t)P->Nmax * (per_slice + per_scratch) <= avail) {
      // everything resident: one segment formed in one pass
      P->seg_len = P->echunk = P->Nmax;
    } else if ((size_t)P->Nmax * per_slice + (size_t)ec_min * per_scratch <= avail) {
      // every propagator resident (no recompute in the backward sweep); the rest holds the
      // Taylor scratch of as many slices as fit
      P->seg_len = P->Nmax;
      P->echunk = (int)std::min<long long>(P->Nmax, (long long)((avail - (size_t)P->Nmax * per_slice) /
                                                                std::max<size_t>(per_scratch, 1)));
    } else {
      // Taylor scratch for a chunk of slices (at most an eighth of the budget, at least 8 slices
      // when they fit), U of as many slices as the rest holds
      long long ec = (long long)(avail / 8 / std::max<size_t>(per_scratch, 1));
      ec = std::max<long long>(1, std::min<long long>(ec, P->Nmax));
      if (ec < 8) ec = std::max<long long>(1, std::min<long long>(8, (long long)(avail / 2 / std::max<size_t>(per_scratch, 1))));
      const size_t left = avail > (size_t)ec * per_scratch ? avail - (size_t)ec * per_scratch : 0;
      const long long seg = (long long)(left / std::max<size_t>(per_slice, 1));
      if (seg < 1 && uplanes > 2) return false;  // the U-only layout may still fit
      // a batch plan that does not fit at all is split into problem groups (its own layout
      // is then never used); a single problem must fit one slice
      QOC_REQUIRE(seg >= 1 || (probs.size() > 1 && !parent), QOC_ERR_OUT_OF_MEMORY,
                  "workspace budget below one slice of propagators");
      const long long seg_ok = std::max<long long>(seg, 1);
      P->seg_len = (int)std::min<long long>(seg_ok, P->Nmax);
      P->echunk = (int)std::min<long long>(ec, P->seg_len);
    }
    P->nseg = (P->Nmax + P->seg_len - 1) / P->seg_len;
    return P->nseg == 1;
  };
  // Room for the gate product tree's second half whenever every propagator stays resident
  // with it (the gate path needs one segment); otherwise U alone, so that longer segments
  // (or every slice) fit.
  P->uplanes = plan_memory(4) ? 4 : 2;
  if (P->uplanes == 2) plan_memory(2);
  const int chunk = P->chunk;
  // layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) / 256 * 256;
    return o;
  };
  P->off_flags = take(256);
  long long njobs_total = 0;
  for (auto& pr : probs) njobs_total += (long long)pr.blocks.size();
  QOC_REQUIRE(njobs_total < (1LL << 30), QOC_ERR_INVALID_ARG, "too many (problem, block) pairs");
  P->entries_per_seg = (long long)P->seg_len * njobs_total;
  P->off_ent = take((size_t)P->entries_per_seg * 16);
  long long tel = 0, ent_off = 0, gacc = 0, u_off = 0, state_base = 0, uout = 0;
  int max_cc = 0;
  long long xw = 0;  // exchange words of the co-operative sweep, per direction
  for (size_t p = 0; p < probs.size(); ++p) {
    const auto& pr = probs[p];
    ProbDev pd{};
    pd.job_begin = (int)P->jobs.size();
    pd.N = pr.N;
    pd.K = pr.sys->K;
    pd.dt = pr.dt;
    pd.u_off = u_off;
    for (auto& b : pr.blocks) {
      JobDev j{};
      j.m = b.m;
      j.mp = b.mp;
      j.d = b.d;
      j.prob = (int)p;
      j.N = pr.N;
      j.K = pr.sys->K;
      j.dt = pr.dt;
      j.h64 = pr.sys->h64.as<double>() + b.h_off;
      j.hT = f64 ? (const void*)(pr.sys->h64.as<double>() + b.h_off) : (const void*)(pr.sys->h32.as<float>() + b.h_off);
      j.pwT = nullptr;
      j.pw_off = -1;
      if (P->pow_free && keeps_products(pr.sys, f64)) {
        j.pwT = f64 ? (const void*)(pr.sys->pw64.as<double>() + pr.sys->pw_off[b.index])
                    : (const void*)(pr.sys->pw32.as<float>() + pr.sys->pw_off[b.index]);
      } else if (P->pow_free) {
        const size_t kidx = std::find(pw_keys.begin(), pw_keys.end(),
                                      std::pair<const qoc_system_s*, int>{pr.sys, b.index}) - pw_keys.begin();
        if (pw_key_off[kidx] < 0) {
          pw_key_off[kidx] = tel;
          tel += (long long)(pair_count(pr.sys->K) + triple_count(pr.sys->K)) * 2 * b.mp * b.mp;
        }
        j.pw_off = pw_key_off[kidx];
      }
      j.state_off = state_base + b.state_off;
      j.u_off = u_off;
      j.ent_off = ent_off;
      ent_off += P->seg_len;
      j.ubuf_off = tel;
      j.uslot = (long long)P->uplanes * b.mp * b.mp;
      tel += (long long)P->seg_len * j.uslot;
      j.sbuf_off = tel;
      tel += (long long)P->echunk * (P->r + 2) * 2 * b.mp * b.mp;
      j.psi_off = tel;
      tel += 2LL * b.mp * (pr.N + 1) * b.d;
      j.lam_off = tel;
      tel += 2LL * b.mp * pr.N * b.d;
      j.cc = (chunk * b.d + 15) / 16 * 16;
      max_cc = std::max(max_cc, j.cc);
      j.gslot = 2LL * b.mp * j.cc;
      j.gbase_off = tel;
      tel += (long long)nslots * j.gslot;
      j.gacc_off = gacc;
      gacc += (long long)j.cc * pr.sys->K;
      j.uout_off = uout;
      uout += (long long)pr.N * b.m * b.m;
      j.xchg_off = xw;
      xw += 2LL * 2 * b.mp * b.d * (f64 ? 2 : 1);
      P->jobs.push_back(j);
    }
    pd.job_end = (int)P->jobs.size();
    P->probs.push_back(pd);
    u_off += (long long)pr.N * pr.sys->K;
    long long D = 0;
    for (auto& b : pr.blocks) D += (long long)b.m * b.d;
    state_base += D;
  }
  P->total_u = u_off;
  P->total_D = state_base;
  P->total_U = uout;
  P->max_cc = max_cc;
  P->off_T = take((size_t)tel * P->elem);
  if (P->pw_ws) {
    if (f64)
      upload_product_descs<double>(P.get(), pw_keys, pw_key_off);
    else
      upload_product_descs<float>(P.get(), pw_keys, pw_key_off);
  }
  P->off_gacc = take((size_t)std::max<long long>(gacc, 1) * 16);
  P->off_sync = take((size_t)2 * 4 * sizeof(int) * P->jobs.size());  // co-operative sweep control words
  P->xchg_words = xw;
  P->off_xchg = take((size_t)2 * xw * 8);  // co-operative sweep state exchange, both directions
  P->bytes = off;
  // panel GEMM descriptors: (job, op) for op = 0..K_job (tiles set by apply_variant)
  for (size_t J = 0; J < P->jobs.size(); ++J)
    for (int o = 0; o <= P->jobs[J].K; ++o) {
      PanelDesc d{};
      d.job = (int)J;
      d.op = o;
      P->panels.push_back(d);
    }
  // device tables (set-up only)
  P->d_jobs.alloc(P->jobs.size() * sizeof(JobDev));
  P->d_probs.alloc(P->probs.size() * sizeof(ProbDev));
  QOC_HIP(hipMemcpy(P->d_probs.ptr, P->probs.data(), P->probs.size() * sizeof(ProbDev), hipMemcpyHostToDevice));
  P->d_panels.alloc(std::max<size_t>(1, P->panels.size()) * sizeof(PanelDesc));
  P->d_theta.alloc(31 * sizeof(double));
  QOC_HIP(hipMemcpy(P->d_theta.ptr, theta, 31 * sizeof(double), hipMemcpyHostToDevice));
  std::vector<double> w((size_t)P->Q * P->Q, 0.0);
  for (int t = 0; t < P->Q; ++t)
    for (int i = 0; i + t < P->Q; ++i) w[(size_t)t * P->Q + i] = fact(i) * fact(t) / fact(i + t + 1);
  P->d_w.alloc(w.size() * sizeof(double));
  QOC_HIP(hipMemcpy(P->d_w.ptr, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice));
  // persistent GEMM grid (resident work-groups, a multiple of the 8 XCDs) and tile tables
  int dev = 0;
  QOC_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  QOC_HIP(hipGetDeviceProperties(&prop, dev));
  const int ncu = prop.multiProcessorCount;
  P->ncu = ncu;
  apply_variant(P.get(), 0);
  // the sweeps keep the state and partial sums in LDS; allow the dynamic size beyond 64 KB
  const int lds = (int)(P->sweep_lds_elems * P->elem);
  // co-operative sweeps when every work-group of a sweep fits on its own CU; the two
  // directions run side by side when both sweeps' work-groups fit together, else one after
  // the other (a plan that segments runs them one after the other anyway)
  {
    const int rb = f64 ? CoopRows<double>::value : CoopRows<float>::value;
    long long groups = 0;
    size_t elems = P->sweep_lds_elems;
    int wmax = 1;
    for (auto& j : P->jobs) {
      const int w = (j.mp + rb - 1) / rb;
      groups += w;
      wmax = std::max(wmax, w);
      elems = std::max(elems, (size_t)2 * j.d * j.mp + (size_t)2 * 16 * j.d * rb);
    }
    P->coop = groups <= ncu && elems * P->elem <= 160 * 1024;
    P->coop_serial = P->coop && 2 * groups > ncu;
    P->coop_w = wmax;
    P->coop_lds = elems * P->elem;
  }
  const int clds = (int)P->coop_lds;
  if (f64) {
    QOC_HIP(hipFuncSetAttribute((const void*)k_sweep<double, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    QOC_HIP(hipFuncSetAttribute((const void*)k_sweep<double, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    QOC_HIP(hipFuncSetAttribute((const void*)k_sweep_coop<double, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, clds));
    QOC_HIP(hipFuncSetAttribute((const void*)k_sweep_coop<double, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, clds));
    QOC_HIP(hipFuncSetAttribute((const void*)k_grad_small<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                96 * 1024));
  } else {
    QOC_HIP(hipFuncSetAttribute((const void*)k_sweep<float, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    QOC_HIP(hipFuncSetAttribute((const void*)k_sweep<float, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    QOC_HIP(hipFuncSetAttribute((const void*)k_sweep_coop<float, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, clds));
    QOC_HIP(hipFuncSetAttribute((const void*)k_sweep_coop<float, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, clds));
    QOC_HIP(hipFuncSetAttribute((const void*)k_grad_small<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                96 * 1024));
  }
  // second stream (default priority) for the backward sweep, and fork/join events
  QOC_HIP(hipStreamCreateWithFlags(&P->st2, hipStreamNonBlocking));
  QOC_HIP(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming));
  QOC_HIP(hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming));
  return P.release();
}

// Bytes a group of problems needs with every propagator resident: states, gradient slots
// for a chunk of `chunk` slices, U of every slice, and the Taylor scratch of
// kGroupChunk slices (the layout build_plan makes, without the alignment of its regions).
// The propagators of a group are formed kGroupChunk slices per round of launches or more:
// a group packed with the scratch of only a few slices would pay each launch's tail many
// times over.
constexpr int kGroupChunk = 32;
static size_t resident_bytes(const std::vector<ProblemSpec>& probs, size_t b0, size_t b1, size_t elem, int r,
                             int nslots, int chunk, bool ws_products) {
  size_t fixed = 0, grad = 0, props = 0, scratch = 0;
  int nmax = 0;
  for (size_t p = b0; p < b1; ++p) nmax = std::max(nmax, probs[p].N);
  for (size_t p = b0; p < b1; ++p) {
    const auto& pr = probs[p];
    for (auto& b : pr.blocks) {
      const size_t mp = (size_t)b.mp;
      fixed += 2 * mp * ((size_t)(pr.N + 1) * b.d + (size_t)pr.N * b.d) * elem;
      const size_t cc = (size_t)(std::min(chunk, nmax) * b.d + 15) / 16 * 16;
      grad += (size_t)nslots * 2 * mp * cc * elem + cc * pr.sys->K * 16;
      props += (size_t)pr.N * 2 * mp * mp * elem;
      if (ws_products && !keeps_products(pr.sys, elem == 8))
        fixed += (size_t)(pair_count(pr.sys->K) + triple_count(pr.sys->K)) * 2 * mp * mp * elem;
      scratch += (size_t)(r + 2) * 2 * mp * mp * elem;
    }
  }
  return fixed + grad + props + (size_t)std::min(nmax, kGroupChunk) * scratch;
}

// Split a batched plan whose propagators do not all fit into groups of consecutive problems
// that do (see qoc_plan_s::groups).  Greedy in problem order by the estimate above; a group
// whose plan still segments is halved, down to single problems, which may segment.
static void group_problems(qoc_plan_s* full, const std::vector<ProblemSpec>& probs, int precision, double u_bound,
                           size_t budget) {
  const int nslots = full->Kmax + 4 + full->R * full->Q;  // the whole batch's series: an upper bound
  const size_t limit = budget / 100 * 97;                  // room for the regions' alignment
  std::vector<std::pair<size_t, size_t>> todo;
  for (size_t b0 = 0; b0 < probs.size();) {
    size_t b1 = b0 + 1;
    while (b1 < probs.size() &&
           resident_bytes(probs, b0, b1 + 1, full->elem, full->r, nslots, std::min(full->Nmax, 2048), full->pw_mode == 2) <=
               limit)
      ++b1;
    todo.push_back({b0, b1});
    b0 = b1;
  }
  std::vector<std::pair<size_t, qoc_plan_s*>> made;
  while (!todo.empty()) {
    const auto [b0, b1] = todo.front();
    todo.erase(todo.begin());
    std::vector<ProblemSpec> sub(probs.begin() + b0, probs.begin() + b1);
    std::unique_ptr<qoc_plan_s> g(build_plan(sub, precision, u_bound, budget, -1, full));
    if (g->nseg > 1 && b1 - b0 > 1) {
      const size_t mid = b0 + (b1 - b0) / 2;
      todo.insert(todo.begin(), {{b0, mid}, {mid, b1}});
      continue;
    }
    made.push_back({b0, g.release()});
  }
  std::sort(made.begin(), made.end());
  size_t bytes = 0;
  for (auto& [b0, g] : made) {
    full->groups.push_back(g);
    full->grp_prob0.push_back((int)b0);
    bytes = std::max(bytes, g->bytes);
  }
  full->bytes = bytes;
}

// Group g's share of a batched call's concatenated arrays: controls and gradients, panels,
// objective outputs and propagators start at its first problem.
struct GroupOffsets {
  long long u, D, out, U;
};
static GroupOffsets group_offsets(const qoc_plan_s* P, size_t g) {
  const int p0 = P->grp_prob0[g];
  const ProbDev& pb = P->probs[p0];
  const JobDev& jb = P->jobs[pb.job_begin];
  return {pb.u_off, jb.state_off, 8LL * p0, jb.uout_off};
}

// Opt-in progress lines (qoc_set_progress): after each problem group of a grouped call a
// host function queued on the stream reports, once the group's work has finished, which
// problems it covered.
static std::atomic<int> g_progress{0};
struct ProgressNote {
  int g, G, p0, p1;
};
static void progress_note_cb(void* p) {
  std::unique_ptr<ProgressNote> n(static_cast<ProgressNote*>(p));
  std::fprintf(stderr, "[qoc] problem group %d/%d done (problems %d..%d)\n", n->g + 1, n->G, n->p0, n->p1 - 1);
  std::fflush(stderr);
}
static void note_group_done(const qoc_plan_s* P, size_t g, hipStream_t st) {
  if (!g_progress.load(std::memory_order_relaxed)) return;
  const int p1 = g + 1 < P->groups.size() ? P->grp_prob0[g + 1] : P->P;
  std::unique_ptr<ProgressNote> n(new ProgressNote{(int)g, (int)P->groups.size(), P->grp_prob0[g], p1});
  QOC_HIP(hipLaunchHostFunc(st, progress_note_cb, n.get()));
  n.release();  // the host function owns it now
}

// The hot-path calls on a plan, group by group when the plan has problem groups.
static void exec_run(qoc_plan_s* P, const double* u, const void* psi0, const void* psif, double* out, double* grad,
                     char* ws, hipStream_t st) {
  if (!P->groups.empty()) {
    for (size_t g = 0; g < P->groups.size(); ++g) {
      const GroupOffsets o = group_offsets(P, g);
      exec_run(P->groups[g], u + o.u, static_cast<const double2*>(psi0) + o.D, static_cast<const double2*>(psif) + o.D,
               out + o.out, grad + o.u, ws, st);
      note_group_done(P, g, st);
    }
    return;
  }
  if (P->prec == QOC_C128)
    Driver<double>::run(P, u, psi0, psif, out, grad, ws, st);
  else
    Driver<float>::run(P, u, psi0, psif, out, grad, ws, st);
}

static void exec_objective(qoc_plan_s* P, const double* u, const void* psi0, const void* psif, double* out, char* ws,
                           hipStream_t st) {
  if (!P->groups.empty()) {
    for (size_t g = 0; g < P->groups.size(); ++g) {
      const GroupOffsets o = group_offsets(P, g);
      exec_objective(P->groups[g], u + o.u, static_cast<const double2*>(psi0) + o.D,
                     static_cast<const double2*>(psif) + o.D, out + o.out, ws, st);
      note_group_done(P, g, st);
    }
    return;
  }
  if (P->prec == QOC_C128)
    Driver<double>::objective_only(P, u, psi0, psif, out, ws, st);
  else
    Driver<float>::objective_only(P, u, psi0, psif, out, ws, st);
}

static void exec_propagate(qoc_plan_s* P, const double* u, double2* U_out, char* ws, hipStream_t st) {
  if (!P->groups.empty()) {
    for (size_t g = 0; g < P->groups.size(); ++g) {
      const GroupOffsets o = group_offsets(P, g);
      exec_propagate(P->groups[g], u + o.u, U_out + o.U, ws, st);
      note_group_done(P, g, st);
    }
    return;
  }
  if (P->prec == QOC_C128)
    Driver<double>::propagate(P, u, U_out, ws, st);
  else
    Driver<float>::propagate(P, u, U_out, ws, st);
}

// Matrix-core rate probe: every wave runs a chain of 16x16x4 MFMAs of the kind the tiles use
// on register operands (8 independent accumulators, no memory traffic), for `iters` rounds.
template <typename T>
__global__ void __launch_bounds__(256) k_mfma_peak(int iters, T* sink) {
  typedef typename Vec4<T>::type V;
  V acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = V{0, 0, 0, 0};
  const T a = (T)(threadIdx.x + 1) * (T)1e-3, b = (T)(blockIdx.x + 1) * (T)1e-3;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = mfma16(a, b, acc[k]);
  }
  T sum = T(0);
#pragma unroll
  for (int k = 0; k < 8; ++k) sum += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  if (sum == T(-1)) sink[0] = sum;  // never true: keeps the chain alive
}

}  // namespace qoc

using namespace qoc;

extern "C" {

qoc_status qoc_plan_create(qoc_system S, int precision, int N, double dt, double u_bound, size_t max_ws,
                           qoc_plan* out) {
  return guarded([&] {
    QOC_REQUIRE(S && out, QOC_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    *out = build_plan({all_blocks(S, N, dt)}, precision, u_bound, max_ws);
  });
}

qoc_status qoc_plan_create_blocks(qoc_system S, const int* blocks, int nblocks, int precision, int N, double dt,
                                  double u_bound, size_t max_ws, qoc_plan* out) {
  return guarded([&] {
    QOC_REQUIRE(S && blocks && out, QOC_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    const int nb = (int)S->blocks.size();
    QOC_REQUIRE(nblocks >= 1 && nblocks <= nb, QOC_ERR_INVALID_ARG, "nblocks must be in 1..number of blocks");
    ProblemSpec pr{S, N, dt, {}};
    int64_t off = 0;
    for (int i = 0; i < nblocks; ++i) {
      QOC_REQUIRE(blocks[i] >= 0 && blocks[i] < nb, QOC_ERR_INVALID_ARG, "block index out of range");
      for (int k = 0; k < i; ++k) QOC_REQUIRE(blocks[k] != blocks[i], QOC_ERR_INVALID_ARG, "repeated block index");
      qoc_system_s::Block b = S->blocks[blocks[i]];
      b.state_off = off;
      off += (int64_t)b.m * b.d;
      pr.blocks.push_back(b);
    }
    *out = build_plan({pr}, precision, u_bound, max_ws);
  });
}

qoc_status qoc_plan_create_batched(const qoc_system* systems, int P, const int* N, const double* dt, int precision,
                                   double u_bound, size_t max_ws, qoc_plan* out) {
  return guarded([&] {
    QOC_REQUIRE(systems && N && dt && out, QOC_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    QOC_REQUIRE(P >= 1 && P <= 65535, QOC_ERR_INVALID_ARG, "P must be in 1..65535");
    std::vector<ProblemSpec> probs;
    for (int p = 0; p < P; ++p) probs.push_back(all_blocks(systems[p], N[p], dt[p]));
    QOC_REQUIRE(precision == QOC_C128 || precision == QOC_C64, QOC_ERR_INVALID_ARG, "unknown precision");
    const int pmode = prepare_powers(probs, precision == QOC_C128);
    const size_t budget = max_ws ? max_ws : default_budget();
    std::unique_ptr<qoc_plan_s> full(build_plan(probs, precision, u_bound, budget, pmode));
    if ((full->nseg > 1 || full->bytes > budget) && P > 1) group_problems(full.get(), probs, precision, u_bound, budget);
    *out = full.release();
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
    size_t per_slice = 0;
    for (auto& j : P->jobs) per_slice += (size_t)(P->uplanes + (P->r + 2) * 2) * j.mp * j.mp * P->elem;
    // a plan with problem groups reports the execution of the group with the most segments
    const qoc_plan_s* E = P;
    int sweep_groups = P->coop ? P->coop_w : 1;
    for (auto* g : P->groups) {
      if (E == P || g->nseg > E->nseg) E = g;
      sweep_groups = std::max(sweep_groups, g->coop ? g->coop_w : 1);
    }
    int64_t v[22] = {E->seg_len, E->nseg, P->r, (int64_t)P->qmax * P->r, P->Q, P->R, (int64_t)per_slice, P->smax,
                     E->chunk, P->grid_gemm, P->P, (int64_t)P->jobs.size(), P->total_u, P->total_D, P->total_U,
                     P->variant, E->echunk, sweep_groups, (int64_t)std::max<size_t>(1, P->groups.size()),
                     P->pow_free, E->uplanes, P->pw_mode == 2 ? 1 : 0};
    for (int i = 0; i < cap && i < 22; ++i) info[i] = v[i];
  });
}

qoc_status qoc_plan_set_variant(qoc_plan P, int variant) {
  return guarded([&] {
    QOC_REQUIRE(P, QOC_ERR_INVALID_ARG, "null plan");
    QOC_REQUIRE(variant >= 0 && variant < kNumVariants, QOC_ERR_INVALID_ARG, "variant out of range");
    QOC_HIP(hipDeviceSynchronize());
    apply_variant(P, variant);
    for (auto* g : P->groups) apply_variant(g, variant);
  });
}

const char* qoc_variant_name(int precision, int variant) {
  if (variant < 0 || variant >= kNumVariants) return "";
  return precision == QOC_C128 ? kVariants64[variant].name : kVariants32[variant].name;
}

qoc_status qoc_plan_autotune(qoc_plan P, const double* u_dev, void* workspace, size_t ws_bytes, void* stream,
                             int* chosen, double* times_ms) {
  return guarded([&] {
    QOC_REQUIRE(P && u_dev && workspace, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(ws_bytes >= P->bytes, QOC_ERR_OUT_OF_MEMORY, "workspace smaller than the plan requires");
    hipStream_t st = (hipStream_t)stream;
    QOC_HIP(hipStreamSynchronize(st));
    hipEvent_t e0, e1;
    QOC_HIP(hipEventCreate(&e0));
    QOC_HIP(hipEventCreate(&e1));
    // a plan with problem groups is timed on its first group (controls from offset 0)
    qoc_plan_s* T = P->groups.empty() ? P : P->groups[0];
    auto run = [&] {
      if (P->prec == QOC_C128)
        Driver<double>::tune_pass(T, u_dev, (char*)workspace, st);
      else
        Driver<float>::tune_pass(T, u_dev, (char*)workspace, st);
    };
    int best = 0;
    double best_ms = 0.0;
    for (int v = 0; v < kNumVariants; ++v) {
      apply_variant(T, v);
      run();  // warm-up
      double t = 1e300;
      for (int rep = 0; rep < 2; ++rep) {
        QOC_HIP(hipEventRecord(e0, st));
        run();
        QOC_HIP(hipEventRecord(e1, st));
        QOC_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        QOC_HIP(hipEventElapsedTime(&ms, e0, e1));
        t = std::min(t, (double)ms);
      }
      if (times_ms) times_ms[v] = t;
      if (v == 0 || t < best_ms) {
        best = v;
        best_ms = t;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    apply_variant(P, best);
    for (auto* g : P->groups) apply_variant(g, best);
    if (chosen) *chosen = best;
  });
}

qoc_status qoc_propagate(qoc_plan P, const double* u_dev, void* U_out_dev, void* workspace, size_t ws_bytes,
                         void* stream) {
  return guarded([&] {
    QOC_REQUIRE(P && u_dev && U_out_dev && workspace, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(ws_bytes >= P->bytes, QOC_ERR_OUT_OF_MEMORY, "workspace smaller than the plan requires");
    exec_propagate(P, u_dev, (double2*)U_out_dev, (char*)workspace, (hipStream_t)stream);
  });
}

qoc_status qoc_fidelity_grad(qoc_plan P, const double* u_dev, const void* psi0_dev, const void* psif_dev,
                             double* out_dev, double* grad_dev, void* workspace, size_t ws_bytes, void* stream) {
  return guarded([&] {
    QOC_REQUIRE(P && u_dev && psi0_dev && psif_dev && out_dev && grad_dev && workspace, QOC_ERR_INVALID_ARG,
                "null argument");
    QOC_REQUIRE(ws_bytes >= P->bytes, QOC_ERR_OUT_OF_MEMORY, "workspace smaller than the plan requires");
    exec_run(P, u_dev, psi0_dev, psif_dev, out_dev, grad_dev, (char*)workspace, (hipStream_t)stream);
  });
}

qoc_status qoc_fidelity(qoc_plan P, const double* u_dev, const void* psi0_dev, const void* psif_dev,
                        double* out_dev, void* workspace, size_t ws_bytes, void* stream) {
  return guarded([&] {
    QOC_REQUIRE(P && u_dev && psi0_dev && psif_dev && out_dev && workspace, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(ws_bytes >= P->bytes, QOC_ERR_OUT_OF_MEMORY, "workspace smaller than the plan requires");
    exec_objective(P, u_dev, psi0_dev, psif_dev, out_dev, (char*)workspace, (hipStream_t)stream);
  });
}

}  // extern "C"

namespace qoc {
// Device memory of qoc_fidelity_grad_noalloc: a file-scope array that the code object
// brings with it, so the call itself allocates nothing.  Its host-side name is not a device
// address: host code uses only the per-device address from hipGetSymbolAddress.
static __device__ __align__(256) char scratch[QOC_STATIC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static char* g_scratch_ptr[256] = {};

// The calling thread's current device's copy of `scratch`, looked up once per device.
static char* static_scratch() {
  int dev = 0;
  QOC_HIP(hipGetDevice(&dev));
  QOC_REQUIRE(dev >= 0 && dev < 256, QOC_ERR_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    QOC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    QOC_REQUIRE(ptr != nullptr, QOC_ERR_DEVICE, "no device address for the static scratch array");
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  return g_scratch_ptr[dev];
}
}  // namespace qoc

extern "C" {

qoc_status qoc_fidelity_grad_noalloc(qoc_plan P, const double* u_dev, const void* psi0_dev, const void* psif_dev,
                                     double* out_dev, double* grad_dev, void* stream) {
  return guarded([&] {
    QOC_REQUIRE(P && u_dev && psi0_dev && psif_dev && out_dev && grad_dev, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(P->bytes <= (size_t)QOC_STATIC_SCRATCH_BYTES, QOC_ERR_OUT_OF_MEMORY,
                "the plan's workspace (" + std::to_string(P->bytes) + " bytes) exceeds the library's static " +
                    "scratch of " + std::to_string((size_t)QOC_STATIC_SCRATCH_BYTES) +
                    " bytes: create the plan with max_workspace_bytes <= QOC_STATIC_SCRATCH_BYTES");
    exec_run(P, u_dev, psi0_dev, psif_dev, out_dev, grad_dev, static_scratch(), (hipStream_t)stream);
  });
}

qoc_status qoc_plan_read_state(qoc_plan P, int problem, int which, int j, const void* workspace, size_t ws_bytes,
                               void* out_dev, void* stream) {
  return guarded([&] {
    QOC_REQUIRE(P && workspace && out_dev, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(ws_bytes >= P->bytes, QOC_ERR_OUT_OF_MEMORY, "workspace smaller than the plan requires");
    QOC_REQUIRE(problem >= 0 && problem < P->P, QOC_ERR_INVALID_ARG, "problem out of range");
    QOC_REQUIRE(which == 0 || which == 1, QOC_ERR_INVALID_ARG, "which must be 0 (state) or 1 (costate)");
    if (!P->groups.empty()) {  // the group that ran this problem, and its index there
      size_t g = P->groups.size() - 1;
      while (P->grp_prob0[g] > problem) --g;
      problem -= P->grp_prob0[g];
      P = P->groups[g];
    }
    const ProbDev& pb = P->probs[problem];
    QOC_REQUIRE(which == 0 ? (j >= 0 && j <= pb.N) : (j >= 1 && j <= pb.N), QOC_ERR_INVALID_ARG,
                "slice index out of range (states 0..N, costates 1..N)");
    hipStream_t st = (hipStream_t)stream;
    const int nj = pb.job_end - pb.job_begin;
    const dim3 grid(16, (unsigned)std::min(nj, 65535));
    if (P->prec == QOC_C128)
      hipLaunchKernelGGL(k_export_state<double>, grid, dim3(256), 0, st, P->d_jobs.as<JobDev>(), pb.job_begin,
                         pb.job_end, (const char*)workspace, P->off_T, which, j, (double2*)out_dev);
    else
      hipLaunchKernelGGL(k_export_state<float>, grid, dim3(256), 0, st, P->d_jobs.as<JobDev>(), pb.job_begin,
                         pb.job_end, (const char*)workspace, P->off_T, which, j, (double2*)out_dev);
    QOC_HIP(hipGetLastError());
  });
}

qoc_status qoc_plan_set_sweep_mode(qoc_plan P, int mode) {
  return guarded([&] {
    QOC_REQUIRE(P, QOC_ERR_INVALID_ARG, "null plan");
    QOC_REQUIRE(mode >= 0 && mode <= (QOC_SWEEP_SOLO | QOC_SWEEP_TEST_STALL_FWD | QOC_SWEEP_TEST_STALL_BWD),
                QOC_ERR_INVALID_ARG, "unknown sweep mode bits");
    P->sweep_mode = mode;
    for (auto* g : P->groups) g->sweep_mode = mode;
  });
}

qoc_status qoc_plan_set_generator_split(qoc_plan P, int ranges) {
  return guarded([&] {
    QOC_REQUIRE(P, QOC_ERR_INVALID_ARG, "null plan");
    QOC_REQUIRE(ranges >= 0, QOC_ERR_INVALID_ARG, "negative number of column ranges");
    P->gen_split = ranges;
    for (auto* g : P->groups) g->gen_split = ranges;
  });
}

qoc_status qoc_plan_groups(qoc_plan P, int* count, int32_t* prob_begin, int32_t* seg_len, int32_t* nseg, int cap) {
  return guarded([&] {
    QOC_REQUIRE(P && count, QOC_ERR_INVALID_ARG, "null argument");
    const int n = std::max<int>(1, (int)P->groups.size());
    *count = n;
    for (int g = 0; g < n && g < cap; ++g) {
      const qoc_plan_s* G = P->groups.empty() ? P : P->groups[g];
      if (prob_begin) prob_begin[g] = P->groups.empty() ? 0 : P->grp_prob0[g];
      if (seg_len) seg_len[g] = G->seg_len;
      if (nseg) nseg[g] = G->nseg;
    }
  });
}

qoc_status qoc_gate_propagate(qoc_plan P, const double* u_dev, void* K_out_dev, void* workspace, size_t ws_bytes,
                              void* stream) {
  return guarded([&] {
    QOC_REQUIRE(P && u_dev && K_out_dev && workspace, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(ws_bytes >= P->bytes, QOC_ERR_OUT_OF_MEMORY, "workspace smaller than the plan requires");
    QOC_REQUIRE(P->P == 1, QOC_ERR_UNSUPPORTED, "gate propagation takes a one-problem plan");
    QOC_REQUIRE(P->nseg == 1 && P->uplanes == 4, QOC_ERR_UNSUPPORTED,
                "gate propagation needs every propagator of the pulse resident twice over (one segment with room "
                "for the product tree)");
    hipStream_t st = (hipStream_t)stream;
    if (P->prec == QOC_C128)
      Driver<double>::gate(P, u_dev, static_cast<double2*>(K_out_dev), (char*)workspace, st);
    else
      Driver<float>::gate(P, u_dev, static_cast<double2*>(K_out_dev), (char*)workspace, st);
    QOC_HIP(hipGetLastError());
  });
}

qoc_status qoc_gate_fidelity(qoc_plan P, const void* Ka_dev, const void* Kb_dev, double* out_dev, void* workspace,
                             size_t ws_bytes, void* stream) {
  return guarded([&] {
    QOC_REQUIRE(P && Ka_dev && Kb_dev && out_dev && workspace, QOC_ERR_INVALID_ARG, "null argument");
    const int njobs = (int)P->jobs.size();
    QOC_REQUIRE(ws_bytes >= (size_t)njobs * kGateParts * 4 * sizeof(double), QOC_ERR_OUT_OF_MEMORY,
                "workspace smaller than the partial sums");
    QOC_REQUIRE(P->P == 1, QOC_ERR_UNSUPPORTED, "gate fidelity takes a one-problem plan");
    hipStream_t st = (hipStream_t)stream;
    double* part = static_cast<double*>(workspace);
    const JobDev* dj = P->d_jobs.as<JobDev>();
    hipLaunchKernelGGL(k_gate_partial, dim3(kGateParts, (unsigned)std::min(njobs, 65535)), dim3(256), 0, st, dj,
                       njobs, static_cast<const double2*>(Ka_dev), static_cast<const double2*>(Kb_dev), part);
    hipLaunchKernelGGL(k_gate_finish, dim3(1), dim3(64), 0, st, dj, njobs, part, out_dev);
    QOC_HIP(hipGetLastError());
  });
}

qoc_status qoc_measure_mfma_peak(int precision, double* tflops, void* stream) {
  return guarded([&] {
    QOC_REQUIRE(tflops, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(precision == QOC_C128 || precision == QOC_C64, QOC_ERR_INVALID_ARG, "unknown precision");
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    QOC_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    QOC_HIP(hipGetDeviceProperties(&prop, dev));
    const void* fn = precision == QOC_C128 ? (const void*)k_mfma_peak<double> : (const void*)k_mfma_peak<float>;
    int occ = 1;
    QOC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 256, 0));
    const int grid = prop.multiProcessorCount * std::max(1, occ);
    const int iters = 1 << 14;
    DeviceBuffer sink(16);
    hipEvent_t e0, e1;
    QOC_HIP(hipEventCreate(&e0));
    QOC_HIP(hipEventCreate(&e1));
    auto launch = [&] {
      if (precision == QOC_C128)
        hipLaunchKernelGGL(k_mfma_peak<double>, dim3(grid), dim3(256), 0, st, iters, sink.as<double>());
      else
        hipLaunchKernelGGL(k_mfma_peak<float>, dim3(grid), dim3(256), 0, st, iters, sink.as<float>());
    };
    launch();  // warm-up
    QOC_HIP(hipEventRecord(e0, st));
    launch();
    QOC_HIP(hipEventRecord(e1, st));
    QOC_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    QOC_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // 2 * 16 * 16 * 4 flops per MFMA, 8 per round per wave, 4 waves per work-group
    *tflops = (double)grid * 4 * 8 * iters * 2048.0 / (ms * 1e-3) / 1e12;
  });
}

qoc_status qoc_set_products_policy(int policy) {
  return guarded([&] {
    QOC_REQUIRE(policy == 0 || policy == 1, QOC_ERR_INVALID_ARG, "policy must be 0 or 1");
    g_products_policy.store(policy);
  });
}

qoc_status qoc_set_progress(int enable) {
  g_progress.store(enable ? 1 : 0, std::memory_order_relaxed);
  return QOC_OK;
}

qoc_status qoc_profile_begin(int max_launches) {
  return guarded([&] {
    QOC_REQUIRE(max_launches >= 0 && max_launches <= (1 << 22), QOC_ERR_INVALID_ARG, "max_launches out of range");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    const size_t want = (size_t)2 * max_launches;
    while (g_prof.pool.size() < want) {
      hipEvent_t e;
      QOC_HIP(hipEventCreate(&e));
      g_prof.pool.push_back(e);
    }
    g_prof.used = 0;
    g_prof.dropped = 0;
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
    const size_t dropped = g_prof.dropped;
    g_prof.recs.clear();
    g_prof.used = 0;
    g_prof.dropped = 0;
    QOC_REQUIRE(dropped == 0, QOC_ERR_INVALID_ARG,
                "more launches than qoc_profile_begin's max_launches: the totals would be partial");
  });
}

qoc_status qoc_plan_slice_stats(qoc_plan P, const double* u_dev, int32_t* q_host, int32_t* s_host, double* norm_host,
                                void* stream) {
  return guarded([&] {
    QOC_REQUIRE(P && u_dev && q_host && s_host && norm_host, QOC_ERR_INVALID_ARG, "null argument");
    hipStream_t st = (hipStream_t)stream;
    const int njobs = (int)P->jobs.size();
    const size_t cnt = (size_t)njobs * P->Nmax;
    DeviceBuffer q(cnt * 4), sbuf(cnt * 4), nrm(cnt * 8);
    hipLaunchKernelGGL(k_slice_norms, dim3(P->Nmax, std::min(njobs, 32768)), dim3(256), 0, st, P->d_jobs.as<JobDev>(), njobs, u_dev,
                       P->Nmax, P->d_theta.as<double>(), P->r, P->qmax, P->t12, P->pow_free, q.as<int>(),
                       sbuf.as<int>(), nrm.as<double>());
    QOC_HIP(hipGetLastError());
    QOC_HIP(hipMemcpyAsync(q_host, q.ptr, cnt * 4, hipMemcpyDeviceToHost, st));
    QOC_HIP(hipMemcpyAsync(s_host, sbuf.ptr, cnt * 4, hipMemcpyDeviceToHost, st));
    QOC_HIP(hipMemcpyAsync(norm_host, nrm.ptr, cnt * 8, hipMemcpyDeviceToHost, st));
    QOC_HIP(hipStreamSynchronize(st));
  });
}

}  // extern "C"
