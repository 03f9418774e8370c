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
// per slice and qubit (n down to 1, the rightmost factor acting first) one pass multiplies
// by the coupling phase and applies the qubit's 2 x 2 factor, then a barrier.  The 2 x 2
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

__global__ void __launch_bounds__(1024) k_lts_apply(int n, const double2* g, LtsPhases ph, int N,
                                                    const double2* in, long long ldin, double2* out) {
  extern __shared__ double2 st[];
  const int D = 1 << n;
  const unsigned mask = (unsigned)D - 1u;
  const int col = blockIdx.x;
  for (int x = threadIdx.x; x < D; x += blockDim.x)
    st[x] = in ? in[(long long)col * ldin + x] : make_double2(x == col ? 1.0 : 0.0, 0.0);
  __syncthreads();
  const int half = D >> 1;
  for (int j = 0; j < N; ++j) {
    for (int i = n; i >= 1; --i) {
      const int p = n - i;
      const double2* f = g + 4 * ((long long)j * n + (i - 1));
      const double2 g00 = f[0], g01 = f[1], g10 = f[2], g11 = f[3];
      for (int t = threadIdx.x; t < half; t += blockDim.x) {
        const unsigned lo = (unsigned)t & ((1u << p) - 1u);
        const unsigned a = (((unsigned)t >> p) << (p + 1)) | lo, b = a | (1u << p);
        const unsigned ra = ((a << 1) | (a >> (n - 1))) & mask, rb = ((b << 1) | (b >> (n - 1))) & mask;
        const double2 va = cmul(st[a], ph.v[__popc(a ^ ra)]), vb = cmul(st[b], ph.v[__popc(b ^ rb)]);
        const double2 na = cmul(g00, va), nb = cmul(g01, vb), ma = cmul(g10, va), mb = cmul(g11, vb);
        st[a] = make_double2(na.x + nb.x, na.y + nb.y);
        st[b] = make_double2(ma.x + mb.x, ma.y + mb.y);
      }
      __syncthreads();
    }
  }
  for (int x = threadIdx.x; x < D; x += blockDim.x) out[(long long)col * D + x] = st[x];
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
    const int threads = std::min(1024, std::max(64, (D / 2 + 63) / 64 * 64));
    hipLaunchKernelGGL(k_lts_apply, dim3((unsigned)ncols), dim3(threads), lds, st, n, g, ph, N,
                       static_cast<const double2*>(psi_in_dev), (long long)D, static_cast<double2*>(psi_out_dev));
    QOC_HIP(hipGetLastError());
  });
}
