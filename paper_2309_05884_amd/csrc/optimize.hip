// GRAPE pulse optimisation: limited-memory BFGS ascent on F(u) (Sec. I; App. B), every
// objective and gradient evaluated by qoc_fidelity_grad, the direction, trial point and
// pair updates by the kernels below (FP64, fixed-order reductions, so a run is
// reproducible).  The line search decides on the host from the eight objective words of
// each trial.
//
// Rule (the paper's own update rule is in its Supplementary Material, not available):
// L-BFGS (Nocedal 1980; Liu & Nocedal 1989) on f = -F with a backtracking Armijo search.
//   d = H g by the two-loop recursion over the last M kept pairs, H0 = gamma I with
//   gamma = s.y / y.y of the newest pair; with no pair, d = (step0 / max|g|) g.
//   A pair s = u_new - u_old, y = g_old - g_new is kept when s.y > 1e-10 sqrt(s.s y.y).
//   g.d <= 0 clears the memory.  Trials alpha = 1, 1/2, ... (max_backtrack halvings);
//   accepted when the evaluation is clean (status word 0) and
//   F(u + alpha d) >= F(u) + c1 alpha g.d.
//
// Memory: the pairs live in a ring of M + 1 slots; a new pair is written to the slot
// after the newest before the curvature test, so a rejected pair never overwrites a kept
// one.
#include "qoc_internal.h"

#include <algorithm>
#include <cmath>

namespace qoc {
namespace {

constexpr int kOptThreads = 1024;
constexpr double kCurvatureEps = 1e-10;

// Sum (or max) over the work-group in a fixed order: each thread's strided partial, then a
// pairwise tree in LDS.  Every thread returns the result.
template <bool MAX>
__device__ double wg_reduce(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = kOptThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      const double a = red[threadIdx.x], b = red[threadIdx.x + h];
      red[threadIdx.x] = MAX ? fmax(a, b) : a + b;
    }
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ double wg_dot(const double* a, const double* b, long long L, double* red) {
  double s = 0.0;
  for (long long i = threadIdx.x; i < L; i += kOptThreads) s += a[i] * b[i];
  return wg_reduce<false>(s, red);
}

// Pair statistics per slot: [0] s.y, [1] y.y, [2] s.s.
// Direction d = H g (or the scaled gradient when count = 0); scal[0] = g.d, scal[1] = max|g|.
// One work-group; thread t owns elements t, t + 1024, ... of every vector, so the vector
// updates need no barrier beyond the reductions'.
__global__ void __launch_bounds__(kOptThreads) k_opt_direction(const double* g, const double* S, const double* Y,
                                                                const double* pst, long long L, int slots,
                                                                int count, int newest, double step0, double* d,
                                                                double* scal) {
  __shared__ double red[kOptThreads];
  __shared__ double alpha[65];
  double gm = 0.0;
  for (long long i = threadIdx.x; i < L; i += kOptThreads) gm = fmax(gm, fabs(g[i]));
  const double gmax = wg_reduce<true>(gm, red);
  if (count == 0) {
    const double c = step0 / gmax;
    for (long long i = threadIdx.x; i < L; i += kOptThreads) d[i] = c * g[i];
  } else {
    for (long long i = threadIdx.x; i < L; i += kOptThreads) d[i] = g[i];
    for (int t = 0; t < count; ++t) {  // newest to oldest
      const int idx = (newest - t + slots) % slots;
      const double* s = S + (size_t)idx * L;
      const double* y = Y + (size_t)idx * L;
      const double a = wg_dot(s, d, L, red) / pst[3 * idx];
      if (threadIdx.x == 0) alpha[t] = a;
      for (long long i = threadIdx.x; i < L; i += kOptThreads) d[i] = d[i] - a * y[i];
    }
    const double gamma = pst[3 * newest] / pst[3 * newest + 1];
    for (long long i = threadIdx.x; i < L; i += kOptThreads) d[i] = gamma * d[i];
    __syncthreads();  // alpha[] written by thread 0 above
    for (int t = count - 1; t >= 0; --t) {  // oldest to newest
      const int idx = (newest - t + slots) % slots;
      const double* s = S + (size_t)idx * L;
      const double* y = Y + (size_t)idx * L;
      const double b = wg_dot(y, d, L, red) / pst[3 * idx];
      const double ab = alpha[t] - b;
      for (long long i = threadIdx.x; i < L; i += kOptThreads) d[i] = d[i] + ab * s[i];
    }
  }
  const double gd = wg_dot(g, d, L, red);
  if (threadIdx.x == 0) {
    scal[0] = gd;
    scal[1] = gmax;
  }
}

__global__ void k_opt_trial(const double* u, const double* d, double alpha, long long L, double* ut) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < L; i += (long long)gridDim.x * blockDim.x)
    ut[i] = u[i] + alpha * d[i];
}

// Accepted trial: the pair into slot, then u <- ut, g <- gt; pst[slot] = (s.y, y.y, s.s).
__global__ void __launch_bounds__(kOptThreads) k_opt_accept(double* u, double* g, const double* ut,
                                                             const double* gt, long long L, double* S, double* Y,
                                                             double* pst, int slot) {
  __shared__ double red[kOptThreads];
  double* s = S + (size_t)slot * L;
  double* y = Y + (size_t)slot * L;
  double sy = 0.0, yy = 0.0, ss = 0.0;
  for (long long i = threadIdx.x; i < L; i += kOptThreads) {
    const double si = ut[i] - u[i], yi = g[i] - gt[i];
    s[i] = si;
    y[i] = yi;
    u[i] = ut[i];
    g[i] = gt[i];
    sy += si * yi;
    yy += yi * yi;
    ss += si * si;
  }
  sy = wg_reduce<false>(sy, red);
  yy = wg_reduce<false>(yy, red);
  ss = wg_reduce<false>(ss, red);
  if (threadIdx.x == 0) {
    pst[3 * slot] = sy;
    pst[3 * slot + 1] = yy;
    pst[3 * slot + 2] = ss;
  }
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct OptLayout {
  size_t plan_bytes = 0, off = 0, total = 0;
  long long L = 0;
  int slots = 0;
  size_t o_ut, o_g, o_gt, o_d, o_S, o_Y, o_pst, o_scal, o_out;
};

// the optimiser's vectors after `base` bytes that the objective uses
OptLayout layout_after(size_t base, long long L, int memory) {
  OptLayout Lo;
  Lo.plan_bytes = base;
  Lo.L = L;
  Lo.slots = memory + 1;
  const size_t vec = align256((size_t)Lo.L * sizeof(double));
  size_t o = align256(base);
  Lo.off = o;
  Lo.o_ut = o; o += vec;
  Lo.o_g = o; o += vec;
  Lo.o_gt = o; o += vec;
  Lo.o_d = o; o += vec;
  Lo.o_S = o; o += vec * Lo.slots;
  Lo.o_Y = o; o += vec * Lo.slots;
  Lo.o_pst = o; o += align256(sizeof(double) * 3 * Lo.slots);
  Lo.o_scal = o; o += 256;
  Lo.o_out = o; o += 256;  // objective words of the current point [0..7] and of the trial [8..15]
  Lo.total = o;
  return Lo;
}

OptLayout opt_layout(qoc_plan plan, int memory) {
  int64_t info[17] = {};
  if (qoc_plan_info(plan, info, 17) != QOC_OK) throw Failure{QOC_ERR_INVALID_ARG, "qoc_plan_info failed"};
  QOC_REQUIRE(info[10] == 1, QOC_ERR_UNSUPPORTED, "the optimiser takes a one-problem plan");
  size_t pb = 0;
  if (qoc_plan_workspace_size(plan, &pb) != QOC_OK) throw Failure{QOC_ERR_INVALID_ARG, "qoc_plan_workspace_size failed"};
  return layout_after(pb, info[12], memory);
}

OptLayout lts_opt_layout(int n, int N, int memory) {
  size_t lb = 0;
  const qoc_status s = qoc_lts_grad_workspace_size(n, N, 1, &lb);
  if (s != QOC_OK) throw Failure{s, std::string("qoc_lts_grad_workspace_size: ") + qoc_last_error()};
  return layout_after(lb, (long long)N * 2 * n, memory);
}

void check_options(const qoc_lbfgs_options* opt) {
  QOC_REQUIRE(opt->max_iter >= 0, QOC_ERR_INVALID_ARG, "max_iter must be >= 0");
  QOC_REQUIRE(opt->memory >= 1 && opt->memory <= 64, QOC_ERR_INVALID_ARG, "memory must be in 1..64");
  QOC_REQUIRE(std::isfinite(opt->step0) && opt->step0 > 0.0, QOC_ERR_INVALID_ARG, "step0 must be positive");
  QOC_REQUIRE(opt->c1 > 0.0 && opt->c1 < 1.0, QOC_ERR_INVALID_ARG, "c1 must be in (0, 1)");
  QOC_REQUIRE(opt->max_backtrack >= 0 && opt->max_backtrack <= 60, QOC_ERR_INVALID_ARG,
              "max_backtrack must be in 0..60");
  QOC_REQUIRE(!std::isnan(opt->f_target) && !std::isnan(opt->gtol), QOC_ERR_INVALID_ARG, "NaN option");
}

}  // namespace
}  // namespace qoc

using namespace qoc;

qoc_status qoc_optimize_workspace_size(qoc_plan plan, int memory, size_t* bytes) {
  return guarded([&] {
    QOC_REQUIRE(plan && bytes, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(memory >= 1 && memory <= 64, QOC_ERR_INVALID_ARG, "memory must be in 1..64");
    *bytes = opt_layout(plan, memory).total;
  });
}

// The L-BFGS iterations of the header, on the controls u_dev (L doubles), with the
// objective and gradient from objective(u, out_dev[8], grad_dev[L]) (asynchronous on
// `stream`); the optimiser's vectors live in `workspace` at the offsets of Lo.
template <class Objective>
void run_lbfgs(const qoc_lbfgs_options* opt, double* u_dev, void* workspace, const OptLayout& Lo, void* stream,
               double* hist_host, int hist_cap, qoc_lbfgs_result* result, Objective&& objective) {
  hipStream_t st = (hipStream_t)stream;
  char* ws = static_cast<char*>(workspace);
  double* ut = reinterpret_cast<double*>(ws + Lo.o_ut);
  double* g = reinterpret_cast<double*>(ws + Lo.o_g);
  double* gt = reinterpret_cast<double*>(ws + Lo.o_gt);
  double* d = reinterpret_cast<double*>(ws + Lo.o_d);
  double* S = reinterpret_cast<double*>(ws + Lo.o_S);
  double* Y = reinterpret_cast<double*>(ws + Lo.o_Y);
  double* pst = reinterpret_cast<double*>(ws + Lo.o_pst);
  double* scal = reinterpret_cast<double*>(ws + Lo.o_scal);
  double* out = reinterpret_cast<double*>(ws + Lo.o_out);
  const long long L = Lo.L;
  const int tgrid = (int)std::min<long long>((L + 255) / 256, 1024);

  // objective words of one evaluation, copied to the host
  auto evaluate = [&](const double* u, double* o_dev, double* grad, double* o_host) {
    objective(u, o_dev, grad);
    QOC_HIP(hipMemcpyAsync(o_host, o_dev, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
    QOC_HIP(hipStreamSynchronize(st));
    const int flags = (int)o_host[7];
    QOC_REQUIRE(!(flags & 4), QOC_ERR_NUMERIC, "a co-operative sweep stalled during the optimisation");
    return flags == 0 && std::isfinite(o_host[0]);
  };
  auto fetch_scal = [&](double* h, int n) {
    QOC_HIP(hipMemcpyAsync(h, scal, n * sizeof(double), hipMemcpyDeviceToHost, st));
    QOC_HIP(hipStreamSynchronize(st));
  };

  double cur[8], trial[8], sc[4];
  QOC_REQUIRE(evaluate(u_dev, out, g, cur), QOC_ERR_NUMERIC,
              "the starting controls give a flagged evaluation (outside the plan's norm bound or non-finite)");
  double F = cur[0];
  int nh = 0, evals = 1, iters = 0, reason = QOC_OPT_MAX_ITER;
  if (nh < hist_cap) hist_host[nh++] = F;
  int count = 0, newest = 0;
  bool stopped = false;
  for (int it = 0; it < opt->max_iter; ++it) {
    if (F >= opt->f_target) {
      reason = QOC_OPT_TARGET;
      stopped = true;
      break;
    }
    hipLaunchKernelGGL(k_opt_direction, dim3(1), dim3(kOptThreads), 0, st, g, S, Y, pst, L, Lo.slots, count,
                       newest, opt->step0, d, scal);
    QOC_HIP(hipGetLastError());
    fetch_scal(sc, 2);
    if (sc[1] <= opt->gtol) {
      reason = QOC_OPT_GTOL;
      stopped = true;
      break;
    }
    if (!(sc[0] > 0.0) && count > 0) {  // not an ascent direction: clear the memory
      count = 0;
      hipLaunchKernelGGL(k_opt_direction, dim3(1), dim3(kOptThreads), 0, st, g, S, Y, pst, L, Lo.slots, 0,
                         newest, opt->step0, d, scal);
      QOC_HIP(hipGetLastError());
      fetch_scal(sc, 2);
    }
    const double gd = sc[0];
    double alpha = 1.0;
    bool accepted = false;
    for (int b = 0; b <= opt->max_backtrack; ++b) {
      hipLaunchKernelGGL(k_opt_trial, dim3(tgrid), dim3(256), 0, st, u_dev, d, alpha, L, ut);
      QOC_HIP(hipGetLastError());
      const bool ok = evaluate(ut, out + 8, gt, trial);
      ++evals;
      if (ok && trial[0] >= F + opt->c1 * alpha * gd) {
        accepted = true;
        break;
      }
      alpha *= 0.5;
    }
    if (!accepted) {
      reason = QOC_OPT_LINE_SEARCH_FAILED;
      stopped = true;
      break;
    }
    const int slot = count == 0 ? 0 : (newest + 1) % Lo.slots;
    hipLaunchKernelGGL(k_opt_accept, dim3(1), dim3(kOptThreads), 0, st, u_dev, g, ut, gt, L, S, Y, pst, slot);
    QOC_HIP(hipGetLastError());
    double ps[3];
    QOC_HIP(hipMemcpyAsync(ps, pst + 3 * slot, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    QOC_HIP(hipStreamSynchronize(st));
    if (ps[0] > kCurvatureEps * std::sqrt(ps[2] * ps[1])) {
      newest = slot;
      count = std::min(count + 1, opt->memory);
    }
    F = trial[0];
    ++iters;
    if (nh < hist_cap) hist_host[nh++] = F;
  }
  if (!stopped && F >= opt->f_target) reason = QOC_OPT_TARGET;
  result->iterations = iters;
  result->evaluations = evals;
  result->reason = reason;
  result->F = F;
  result->iterations = iters;
  result->evaluations = evals;
  result->reason = reason;
  result->F = F;
}

qoc_status qoc_optimize_lbfgs(qoc_plan plan, const qoc_lbfgs_options* opt, double* u_dev, const void* psi0_dev,
                              const void* psif_dev, void* workspace, size_t ws_bytes, void* stream,
                              double* hist_host, int hist_cap, qoc_lbfgs_result* result) {
  return guarded([&] {
    QOC_REQUIRE(plan && opt && u_dev && psi0_dev && psif_dev && workspace && result, QOC_ERR_INVALID_ARG,
                "null argument");
    check_options(opt);
    QOC_REQUIRE(hist_cap >= 0 && (hist_cap == 0 || hist_host), QOC_ERR_INVALID_ARG, "bad history buffer");
    const OptLayout Lo = opt_layout(plan, opt->memory);
    QOC_REQUIRE(ws_bytes >= Lo.total, QOC_ERR_OUT_OF_MEMORY, "workspace smaller than qoc_optimize_workspace_size");
    run_lbfgs(opt, u_dev, workspace, Lo, stream, hist_host, hist_cap, result,
              [&](const double* u, double* o_dev, double* grad) {
                const qoc_status s = qoc_fidelity_grad(plan, u, psi0_dev, psif_dev, o_dev, grad, workspace,
                                                       Lo.plan_bytes, stream);
                if (s != QOC_OK) throw Failure{s, std::string("qoc_fidelity_grad: ") + qoc_last_error()};
              });
  });
}

qoc_status qoc_optimize_lts_workspace_size(int n, int N, int memory, size_t* bytes) {
  return guarded([&] {
    QOC_REQUIRE(bytes, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(memory >= 1 && memory <= 64, QOC_ERR_INVALID_ARG, "memory must be in 1..64");
    *bytes = lts_opt_layout(n, N, memory).total;
  });
}

qoc_status qoc_optimize_lbfgs_lts(int n, double Bz, double c_cpl, int N, double dt, const qoc_lbfgs_options* opt,
                                  double* u_dev, const void* psi0_dev, const void* psif_dev, void* workspace,
                                  size_t ws_bytes, void* stream, double* hist_host, int hist_cap,
                                  qoc_lbfgs_result* result) {
  return guarded([&] {
    QOC_REQUIRE(opt && u_dev && psi0_dev && psif_dev && workspace && result, QOC_ERR_INVALID_ARG, "null argument");
    check_options(opt);
    QOC_REQUIRE(hist_cap >= 0 && (hist_cap == 0 || hist_host), QOC_ERR_INVALID_ARG, "bad history buffer");
    const OptLayout Lo = lts_opt_layout(n, N, opt->memory);
    QOC_REQUIRE(ws_bytes >= Lo.total, QOC_ERR_OUT_OF_MEMORY, "workspace smaller than qoc_optimize_lts_workspace_size");
    run_lbfgs(opt, u_dev, workspace, Lo, stream, hist_host, hist_cap, result,
              [&](const double* u, double* o_dev, double* grad) {
                const qoc_status s = qoc_lts_fidelity_grad(n, Bz, c_cpl, u, N, dt, 1, psi0_dev, psif_dev, o_dev, grad,
                                                           workspace, Lo.plan_bytes, stream);
                if (s != QOC_OK) throw Failure{s, std::string("qoc_lts_fidelity_grad: ") + qoc_last_error()};
              });
  });
}
