// Trotterised propagator for per-qubit controls (Sec. III B, Eqs. (8)-(11)), applied to
// state columns on the GPU.
//
// H_j = sum_i [(B_z/2) sz_i + (Bx_i[j] sx_i + By_i[j] sy_i)/2] + (c/4) sum_i sz_i sz_{i+1}
// (ring), U_j^LTS = prod_{i=1..n} [exp(-i dt h_i[j].sigma_i) exp(-i (dt/n) H_cpl)] with
// h_i[j] = (Bx_i[j], By_i[j], B_z) / 2.  Eq. (11) shows that each qubit factor is 2^(n-1)
// copies of one 2 x 2 block once qubit i is swapped to the last place, and that the
// coupling factor is block diagonal under D_n.  On the GPU the swap is an index map: the
// 2 x 2 block acts on the amplitude pairs that differ in qubit i's bit, and the coupling
// is diagonal in the computational basis, a phase that depends only on the number k of
// unequal neighbour pairs on the ring, sum_i z_i z_{i+1} = n - 2k.
//
// One work-group owns one column (2^n amplitudes in LDS, n <= 13) for the whole pulse:
// per slice and qubit (n down to 1, the rightmost factor acting first) the column is
// multiplied by the coupling phase and the qubit's 2 x 2 factor is applied; three qubits
// share one pass over LDS (their 8 amplitudes in registers), then a barrier.  The 2 x 2
// factors of every (slice, qubit) are formed first, in closed form
// exp(-i t h.sigma) = cos(t|h|) I - i sin(t|h|)/|h| h.sigma, by k_lts_factors.  All
// arithmetic is FP64.  Qubit q sits at bit n - q; bit 0 is spin up (z = +1).
#include "qoc_internal.h"

#include <algorithm>
#include <cmath>

namespace qoc {
namespace {

constexpr int kLtsMaxQubits = 13;

struct LtsPhases {
  double2 v[kLtsMaxQubits + 1];  // exp(-i (dt/n) (c/4) (n - 2k)), k = 0..n
};

__global__ void k_lts_factors(int n, double Bz, const double* u, int N, double dt, double2* g) {
  const long long total = (long long)N * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long j = e / n;
    const int i = (int)(e % n);  // qubit i + 1
    const double hx = 0.5 * u[j * 2 * n + 2 * i], hy = 0.5 * u[j * 2 * n + 2 * i + 1], hz = 0.5 * Bz;
    const double r = sqrt(hx * hx + hy * hy + hz * hz);
    const double c = cos(dt * r);
    const double sr = r > 0.0 ? sin(dt * r) / r : dt;
    double2* o = g + 4 * e;
    o[0] = make_double2(c, -sr * hz);       // row 0 (spin up), column 0
    o[1] = make_double2(-sr * hy, -sr * hx);  // row 0, column 1: -i sr (hx - i hy)
    o[2] = make_double2(sr * hy, -sr * hx);   // row 1, column 0: -i sr (hx + i hy)
    o[3] = make_double2(c, sr * hz);          // row 1, column 1
  }
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One LDS pass over Q consecutive qubit bits p .. p + Q - 1 (qubits n - p, n - p - 1, ...,
// applied in that order): each thread takes the 2^Q amplitudes that differ only in those
// bits into registers and applies, per bit, the coupling phase and that qubit's 2 x 2
// factor, so a slice needs ceil(n / 3) passes and barriers instead of n.
template <int Q>
__device__ inline void lts_pass(double2* st, int n, int p, const double2* gj, int es, const LtsPhases& ph) {
  constexpr int M = 1 << Q;
  const int D = 1 << n;
  const unsigned mask = (unsigned)D - 1u;
  double2 g[Q][4];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const double2* f = gj + es * (n - (p + k) - 1);  // qubit n - (p + k); es entries per factor
#pragma unroll
    for (int e = 0; e < 4; ++e) g[k][e] = f[e];
  }
  for (int t = threadIdx.x; t < (D >> Q); t += blockDim.x) {
    const unsigned lo = (unsigned)t & ((1u << p) - 1u);
    const unsigned base = (((unsigned)t >> p) << (p + Q)) | lo;
    double2 v[M], e[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const unsigned a = base | ((unsigned)m << p);
      const unsigned ra = ((a << 1) | (a >> (n - 1))) & mask;
      v[m] = st[a];
      e[m] = ph.v[__popc(a ^ ra)];
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
#pragma unroll
      for (int m = 0; m < M; ++m) v[m] = cmul(v[m], e[m]);
#pragma unroll
      for (int m = 0; m < M; ++m) {
        if (m & (1 << k)) continue;
        const int m1 = m | (1 << k);
        const double2 x0 = v[m], x1 = v[m1];
        const double2 n0 = cmul(g[k][0], x0), n1 = cmul(g[k][1], x1), q0 = cmul(g[k][2], x0), q1 = cmul(g[k][3], x1);
        v[m] = make_double2(n0.x + n1.x, n0.y + n1.y);
        v[m1] = make_double2(q0.x + q1.x, q0.y + q1.y);
      }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) st[base | ((unsigned)m << p)] = v[m];
  }
}

// the slices j of the pulse on the column in st, three qubits per pass; the factors hold
// es entries per (slice, qubit), the 2 x 2 factor first
__device__ inline void lts_forward(double2* st, int n, const double2* g, int N, const LtsPhases& ph, int es) {
  for (int j = 0; j < N; ++j) {
    const double2* gj = g + (long long)es * j * n;
    for (int p = 0; p < n;) {
      const int Q = n - p >= 3 ? 3 : n - p;
      if (Q == 3)
        lts_pass<3>(st, n, p, gj, es, ph);
      else if (Q == 2)
        lts_pass<2>(st, n, p, gj, es, ph);
      else
        lts_pass<1>(st, n, p, gj, es, ph);
      p += Q;
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(1024) k_lts_apply(int n, const double2* g, LtsPhases ph, int N,
                                                    const double2* in, long long ldin, double2* out) {
  extern __shared__ double2 st[];
  const int D = 1 << n;
  const int col = blockIdx.x;
  for (int x = threadIdx.x; x < D; x += blockDim.x)
    st[x] = in ? in[(long long)col * ldin + x] : make_double2(x == col ? 1.0 : 0.0, 0.0);
  __syncthreads();
  lts_forward(st, n, g, N, ph, 4);
  for (int x = threadIdx.x; x < D; x += blockDim.x) out[(long long)col * D + x] = st[x];
}

// The factor and its derivatives for the gradient: per (problem, slice, qubit) twelve
// entries, g then dg/dBx then dg/dBy (row-major 2 x 2 each).  With h = (Bx, By, B_z) / 2,
// r = |h|, s = sin(t r) / r: g = cos(t r) I - i s h.sigma and
//   dg/dh_a = -t sin(t r) (h_a / r) I - i s'(r) (h_a / r) h.sigma - i s sigma_a,
//   s'(r) = (t r cos(t r) - sin(t r)) / r^2,  dg/dB_a = dg/dh_a / 2.
__global__ void k_lts_factors_grad(int n, double Bz, const double* u, long long NP, double dt, double2* g) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < NP * n;
       e += (long long)gridDim.x * blockDim.x) {
    const long long j = e / n;  // slice index over all problems (problem-major)
    const int i = (int)(e % n);
    const double hx = 0.5 * u[j * 2 * n + 2 * i], hy = 0.5 * u[j * 2 * n + 2 * i + 1], hz = 0.5 * Bz;
    const double r = sqrt(hx * hx + hy * hy + hz * hz);
    const double tr = dt * r, c = cos(tr), sn = sin(tr);
    const double s = r > 0.0 ? sn / r : dt;
    // s'(r) / r, with its series where t r is small
    const double spr = tr > 1e-3 ? (tr * c - sn) / (r * r * r) : -dt * dt * dt / 3.0 * (1.0 - tr * tr / 10.0);
    double2* o = g + 12 * e;
    o[0] = make_double2(c, -s * hz);
    o[1] = make_double2(-s * hy, -s * hx);
    o[2] = make_double2(s * hy, -s * hx);
    o[3] = make_double2(c, s * hz);
    const double hs[2] = {hx, hy};
    for (int a = 0; a < 2; ++a) {
      const double A = r > 0.0 ? -dt * sn * hs[a] / r : 0.0, B = spr * hs[a];
      // -i s sigma_a: sigma_x -> (0,1), (1,0) = -i s; sigma_y -> (0,1) = -s, (1,0) = +s
      const double2 sx01 = a == 0 ? make_double2(0.0, -s) : make_double2(-s, 0.0);
      const double2 sx10 = a == 0 ? make_double2(0.0, -s) : make_double2(s, 0.0);
      double2* d = o + 4 + 4 * a;
      d[0] = make_double2(0.5 * A, -0.5 * B * hz);
      d[1] = make_double2(0.5 * (-B * hy + sx01.x), 0.5 * (-B * hx + sx01.y));
      d[2] = make_double2(0.5 * (B * hy + sx10.x), 0.5 * (-B * hx + sx10.y));
      d[3] = make_double2(0.5 * A, 0.5 * B * hz);
    }
  }
}

__device__ inline double2 cconjmul(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// The backward step over Q consecutive qubit bits low .. low + Q - 1, taken from the highest
// bit down (the reverse of the forward order): per bit, the gate is undone on psi, the
// derivative products <lambda| dg/dB_a |psi> are accumulated into d[bit - low], the adjoint
// gate is applied to lambda, then the coupling phase is undone on both; each thread holds
// the 2^Q amplitudes of psi and lambda that differ in those bits.
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

template <int Q>
__device__ inline void lts_back_pass(double2* ps, double2* lm, int n, int low, const double2* Fj,
                                     const LtsPhases& ph, double (&d)[3][4]) {
  constexpr int M = 1 << Q;
  const int D = 1 << n;
  const unsigned mask = (unsigned)D - 1u;
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int q = 0; q < 4; ++q) d[k][q] = 0.0;
  for (int t = threadIdx.x; t < (D >> Q); t += blockDim.x) {
    const unsigned lo = (unsigned)t & ((1u << low) - 1u);
    const unsigned base = (((unsigned)t >> low) << (low + Q)) | lo;
    double2 v[M], l[M], e[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const unsigned a = base | ((unsigned)m << low);
      const unsigned ra = ((a << 1) | (a >> (n - 1))) & mask;
      v[m] = ps[a];
      l[m] = lm[a];
      e[m] = ph.v[__popc(a ^ ra)];
    }
#pragma unroll
    for (int k = Q - 1; k >= 0; --k) {
      const double2* f = Fj + 12 * (n - (low + k) - 1);  // qubit n - (low + k)
      const double2 g00 = f[0], g01 = f[1], g10 = f[2], g11 = f[3];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        if (m & (1 << k)) continue;
        const int m1 = m | (1 << k);
        const double2 p0 = v[m], p1 = v[m1], l0 = l[m], l1 = l[m1];
        const double2 q0 = cadd(cconjmul(g00, p0), cconjmul(g10, p1));
        const double2 q1 = cadd(cconjmul(g01, p0), cconjmul(g11, p1));
        const double2 ax0 = cadd(cmul(f[4], q0), cmul(f[5], q1)), ax1 = cadd(cmul(f[6], q0), cmul(f[7], q1));
        const double2 ay0 = cadd(cmul(f[8], q0), cmul(f[9], q1)), ay1 = cadd(cmul(f[10], q0), cmul(f[11], q1));
        const double2 cx = cadd(cconjmul(l0, ax0), cconjmul(l1, ax1)), cy = cadd(cconjmul(l0, ay0), cconjmul(l1, ay1));
        d[k][0] += cx.x;
        d[k][1] += cx.y;
        d[k][2] += cy.x;
        d[k][3] += cy.y;
        v[m] = q0;
        v[m1] = q1;
        l[m] = cadd(cconjmul(g00, l0), cconjmul(g10, l1));
        l[m1] = cadd(cconjmul(g01, l0), cconjmul(g11, l1));
      }
#pragma unroll
      for (int m = 0; m < M; ++m) {
        v[m] = cconjmul(e[m], v[m]);
        l[m] = cconjmul(e[m], l[m]);
      }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const unsigned a = base | ((unsigned)m << low);
      ps[a] = v[m];
      lm[a] = l[m];
    }
  }
}

// One work-group per problem, state and costate in LDS (n <= 12).  Forward: the pulse on
// psi_0 (three qubits per pass).  Then o, the norms, and backward, factor by factor in
// reverse, two qubits per pass (lts_back_pass): the gate is undone on psi (giving the
// state just before it) and applied adjoint to lambda (the costate just after it becomes
// the one just before it) while the pass accumulates <lambda_after| dg/dB_a |psi_before>
// for a = x, y; the coupling phase is then undone on both.  The wave partials of a pass go
// to one of two LDS slots by parity, so one barrier per pass suffices; thread 0 adds them
// up after that barrier.
__global__ void __launch_bounds__(512) k_lts_grad(int n, const double2* fac, LtsPhases ph, int N,
                                                   const double2* psi0, const double2* psif, double* out,
                                                   double* grad) {
  extern __shared__ double2 sm[];
  __shared__ double part[2][16][12];
  __shared__ double ored[16][4];
  __shared__ double osum[4];
  const int D = 1 << n;
  const int p = blockIdx.x;
  double2* ps = sm;
  double2* lm = sm + D;
  const double2* F = fac + (size_t)p * N * n * 12;
  for (int x = threadIdx.x; x < D; x += blockDim.x) ps[x] = psi0[(size_t)p * D + x];
  __syncthreads();
  lts_forward(ps, n, F, N, ph, 12);
  // o = <psi_f|psi_N>, norms
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  {
    double orr = 0.0, oii = 0.0, nN = 0.0, nf = 0.0;
    for (int x = threadIdx.x; x < D; x += blockDim.x) {
      const double2 l = psif[(size_t)p * D + x], v = ps[x];
      lm[x] = l;
      const double2 c = cconjmul(l, v);
      orr += c.x;
      oii += c.y;
      nN += v.x * v.x + v.y * v.y;
      nf += l.x * l.x + l.y * l.y;
    }
    double vals[4] = {orr, oii, nN, nf};
    for (int q = 0; q < 4; ++q) {
      double v = vals[q];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) ored[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
      double v = 0.0;
      for (int w = 0; w < nw; ++w) v += ored[w][threadIdx.x];
      osum[threadIdx.x] = v;
    }
    __syncthreads();
  }
  const double o_r = osum[0], o_i = osum[1], nN = osum[2], nf = osum[3];
  if (threadIdx.x == 0) {
    double* o = out + (size_t)p * 8;
    const double raw = o_r * o_r + o_i * o_i;
    o[0] = raw / (nN * nf);
    o[1] = raw;
    o[2] = o_r;
    o[3] = o_i;
    o[4] = nN;
    o[5] = nf;
    o[6] = 0.0;
    o[7] = isfinite(o[0]) ? 0.0 : 2.0;
  }
  const double scale = 2.0 / (nN * nf);
  double* G = grad + (size_t)p * N * 2 * n;
  int step = 0;
  for (int j = N - 1; j >= 0; --j)
    for (int top = n - 1; top >= 0;) {  // bits top, top - 1, ... (qubits 1, 2, ...), two per pass
      const int Q = top >= 1 ? 2 : 1;
      const int low = top - Q + 1;
      double d[3][4];
      if (Q == 2)
        lts_back_pass<2>(ps, lm, n, low, F + 12 * (size_t)j * n, ph, d);
      else
        lts_back_pass<1>(ps, lm, n, low, F + 12 * (size_t)j * n, ph, d);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (k >= Q) break;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double v = d[k][q];
          for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
          if (lane == 0) part[step & 1][wave][4 * k + q] = v;
        }
      }
      __syncthreads();
      if (threadIdx.x == 0)
        for (int k = 0; k < Q; ++k) {
          double s4[4] = {0.0, 0.0, 0.0, 0.0};
          for (int w = 0; w < nw; ++w)
            for (int q = 0; q < 4; ++q) s4[q] += part[step & 1][w][4 * k + q];
          const int i = n - (low + k);  // qubit of bit low + k
          // 2 Re(conj(o) d) / norms
          G[(size_t)j * 2 * n + 2 * (i - 1)] = scale * (o_r * s4[0] + o_i * s4[1]);
          G[(size_t)j * 2 * n + 2 * (i - 1) + 1] = scale * (o_r * s4[2] + o_i * s4[3]);
        }
      ++step;
      top -= Q;
    }
}

}  // namespace
}  // namespace qoc

using namespace qoc;

qoc_status qoc_lts_workspace_size(int n, int N, size_t* bytes) {
  return guarded([&] {
    QOC_REQUIRE(bytes, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(n >= 1 && n <= kLtsMaxQubits, QOC_ERR_UNSUPPORTED, "n must be in 1..13 (the column lives in LDS)");
    QOC_REQUIRE(N >= 1, QOC_ERR_INVALID_ARG, "N must be >= 1");
    *bytes = (size_t)N * n * 4 * sizeof(double2);
  });
}

qoc_status qoc_lts_apply(int n, double Bz, double c_cpl, const double* u_dev, int N, double dt, const void* psi_in_dev,
                         int ncols, void* psi_out_dev, void* workspace, size_t ws_bytes, void* stream) {
  return guarded([&] {
    QOC_REQUIRE(u_dev && psi_out_dev && workspace, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(n >= 1 && n <= kLtsMaxQubits, QOC_ERR_UNSUPPORTED, "n must be in 1..13 (the column lives in LDS)");
    QOC_REQUIRE(N >= 1 && N <= (1 << 26), QOC_ERR_INVALID_ARG, "N must be in 1..2^26");
    QOC_REQUIRE(std::isfinite(Bz) && std::isfinite(c_cpl) && std::isfinite(dt) && dt > 0.0, QOC_ERR_INVALID_ARG,
                "B_z, c_cpl and dt must be finite, dt > 0");
    const int D = 1 << n;
    QOC_REQUIRE(ncols >= 1 && (psi_in_dev || ncols <= D), QOC_ERR_INVALID_ARG,
                "ncols must be >= 1 (at most 2^n for identity columns)");
    QOC_REQUIRE(ncols <= (1 << 24), QOC_ERR_INVALID_ARG, "ncols must be at most 2^24");
    QOC_REQUIRE(ws_bytes >= (size_t)N * n * 4 * sizeof(double2), QOC_ERR_OUT_OF_MEMORY,
                "workspace smaller than qoc_lts_workspace_size");
    hipStream_t st = (hipStream_t)stream;
    double2* g = static_cast<double2*>(workspace);
    const long long nf = (long long)N * n;
    hipLaunchKernelGGL(k_lts_factors, dim3((unsigned)std::min<long long>((nf + 255) / 256, 4096)), dim3(256), 0, st,
                       n, Bz, u_dev, N, dt, g);
    QOC_HIP(hipGetLastError());
    LtsPhases ph{};
    for (int k = 0; k <= n; ++k) {
      const double a = -(dt / n) * 0.25 * c_cpl * (double)(n - 2 * k);
      ph.v[k] = make_double2(std::cos(a), std::sin(a));
    }
    const int lds = D * (int)sizeof(double2);
    QOC_HIP(hipFuncSetAttribute((const void*)k_lts_apply, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    const int threads = std::min(1024, std::max(64, (D / 8 + 63) / 64 * 64));
    hipLaunchKernelGGL(k_lts_apply, dim3((unsigned)ncols), dim3(threads), lds, st, n, g, ph, N,
                       static_cast<const double2*>(psi_in_dev), (long long)D, static_cast<double2*>(psi_out_dev));
    QOC_HIP(hipGetLastError());
  });
}

qoc_status qoc_lts_grad_workspace_size(int n, int N, int P, size_t* bytes) {
  return guarded([&] {
    QOC_REQUIRE(bytes, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(n >= 1 && n <= kLtsMaxQubits - 1, QOC_ERR_UNSUPPORTED,
                "n must be in 1..12 (state and costate live in LDS)");
    QOC_REQUIRE(N >= 1 && P >= 1, QOC_ERR_INVALID_ARG, "N and P must be >= 1");
    *bytes = (size_t)P * N * n * 12 * sizeof(double2);
  });
}

qoc_status qoc_lts_fidelity_grad(int n, double Bz, double c_cpl, const double* u_dev, int N, double dt, int P,
                                 const void* psi0_dev, const void* psif_dev, double* out_dev, double* grad_dev,
                                 void* workspace, size_t ws_bytes, void* stream) {
  return guarded([&] {
    QOC_REQUIRE(u_dev && psi0_dev && psif_dev && out_dev && grad_dev && workspace, QOC_ERR_INVALID_ARG,
                "null argument");
    QOC_REQUIRE(n >= 1 && n <= kLtsMaxQubits - 1, QOC_ERR_UNSUPPORTED,
                "n must be in 1..12 (state and costate live in LDS)");
    QOC_REQUIRE(N >= 1 && N <= (1 << 26) && P >= 1 && P <= 65535, QOC_ERR_INVALID_ARG,
                "N must be in 1..2^26 and P in 1..65535");
    QOC_REQUIRE(std::isfinite(Bz) && std::isfinite(c_cpl) && std::isfinite(dt) && dt > 0.0, QOC_ERR_INVALID_ARG,
                "B_z, c_cpl and dt must be finite, dt > 0");
    QOC_REQUIRE(ws_bytes >= (size_t)P * N * n * 12 * sizeof(double2), QOC_ERR_OUT_OF_MEMORY,
                "workspace smaller than qoc_lts_grad_workspace_size");
    hipStream_t st = (hipStream_t)stream;
    double2* g = static_cast<double2*>(workspace);
    const long long NP = (long long)N * P;
    hipLaunchKernelGGL(k_lts_factors_grad, dim3((unsigned)std::min<long long>((NP * n + 255) / 256, 4096)),
                       dim3(256), 0, st, n, Bz, u_dev, NP, dt, g);
    QOC_HIP(hipGetLastError());
    LtsPhases ph{};
    for (int k = 0; k <= n; ++k) {
      const double a = -(dt / n) * 0.25 * c_cpl * (double)(n - 2 * k);
      ph.v[k] = make_double2(std::cos(a), std::sin(a));
    }
    const int D = 1 << n;
    const int lds = 2 * D * (int)sizeof(double2);
    QOC_HIP(hipFuncSetAttribute((const void*)k_lts_grad, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    const int threads = std::min(512, std::max(64, (D / 4 + 63) / 64 * 64));
    hipLaunchKernelGGL(k_lts_grad, dim3((unsigned)P), dim3(threads), lds, st, n, g, ph, N,
                       static_cast<const double2*>(psi0_dev), static_cast<const double2*>(psif_dev), out_dev,
                       grad_dev);
    QOC_HIP(hipGetLastError());
  });
}
