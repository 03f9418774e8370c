// Projection of Pauli-sum Hamiltonians into the symmetry-adapted blocks
// (Sec. II A and Fig. 2: A^dag H A is block diagonal; App. A for the bases).
//
// For a one-dimensional irrep chi the block entry between representatives b, a is
//     <b,chi|H|a,chi> = sqrt(|O_a| / |O_b|) * sum_{x in O_b} H[x,a] chi(g_x),   g_x b = x,
// which follows from H commuting with the group: the image H|a> is canonicalised
// term by term.  Momentum blocks use the same formula with the rotation subgroup and
// chi_k(rho^l) = exp(i k l).  One thread owns one column (one representative a), so
// every entry is accumulated by exactly one thread in a fixed order: no atomics and
// bit-reproducible sums.  The symmetric group uses the |J,M> closed form on the host.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cctype>
#include <map>

#include "bits.h"
#include "qoc_internal.h"

namespace qoc {

// ------------------------------------------------------------------- term expansion
static int op_bits(char a, uint64_t& x, uint64_t& z, int p) {
  switch (a) {
    case 'x': case 'X': x |= 1ull << p; return 0;
    case 'y': case 'Y': x |= 1ull << p; z |= 1ull << p; return 0;
    case 'z': case 'Z': z |= 1ull << p; return 0;
    default: return -1;
  }
}

static bool site_selected(int sites, int q) {
  if (sites == QOC_SITES_ALL) return true;
  if (sites == QOC_SITES_EVEN) return q % 2 == 0;
  if (sites == QOC_SITES_ODD) return q % 2 == 1;
  return false;
}

// Expand terms into Pauli strings on bit positions (qubit q -> position n - q) and merge
// equal strings.  Every site of a string carries one Pauli factor, so products of
// factors on distinct sites need no reordering phase.
std::vector<PauliString> expand_terms(int n, const qoc_term* terms, int count) {
  QOC_REQUIRE(count >= 0 && (count == 0 || terms), QOC_ERR_INVALID_ARG, "null term array");
  std::map<std::pair<uint64_t, uint64_t>, double> acc;
  auto add = [&](uint64_t x, uint64_t z, double c) { acc[{x, z}] += c; };
  for (int t = 0; t < count; ++t) {
    const qoc_term& T = terms[t];
    QOC_REQUIRE(std::isfinite(T.coeff), QOC_ERR_INVALID_ARG, "non-finite term coefficient");
    switch (T.kind) {
      case QOC_TERM_ONE_BODY: {
        QOC_REQUIRE(T.sites >= 0 && T.sites <= 2, QOC_ERR_INVALID_ARG, "bad site selection");
        for (int q = 1; q <= n; ++q) {
          if (!site_selected(T.sites, q)) continue;
          uint64_t x = 0, z = 0;
          QOC_REQUIRE(op_bits(T.op_a, x, z, n - q) == 0, QOC_ERR_INVALID_ARG, "bad Pauli letter");
          double w = (T.staggered && (q % 2)) ? -1.0 : 1.0;
          add(x, z, T.coeff * w);
        }
        break;
      }
      case QOC_TERM_RING_PAIR: {
        QOC_REQUIRE(T.distance % n != 0, QOC_ERR_INVALID_ARG, "ring pair distance is 0 mod n");
        for (int q = 1; q <= n; ++q) {
          int q2 = ((q - 1 + T.distance) % n + n) % n + 1;
          uint64_t x = 0, z = 0, x2 = 0, z2 = 0;
          QOC_REQUIRE(op_bits(T.op_a, x, z, n - q) == 0 && op_bits(T.op_b, x2, z2, n - q2) == 0,
                      QOC_ERR_INVALID_ARG, "bad Pauli letter");
          add(x | x2, z | z2, T.coeff);
        }
        break;
      }
      case QOC_TERM_ALL_PAIRS: {
        for (int q = 1; q <= n; ++q)
          for (int q2 = q + 1; q2 <= n; ++q2) {
            uint64_t x = 0, z = 0, x2 = 0, z2 = 0;
            QOC_REQUIRE(op_bits(T.op_a, x, z, n - q) == 0 && op_bits(T.op_b, x2, z2, n - q2) == 0,
                        QOC_ERR_INVALID_ARG, "bad Pauli letter");
            add(x | x2, z | z2, T.coeff);
          }
        break;
      }
      case QOC_TERM_PAULI_STRING: {
        QOC_REQUIRE(((T.x_mask | T.z_mask) & ~nmask(n)) == 0, QOC_ERR_INVALID_ARG, "Pauli mask beyond n bits");
        add(T.x_mask, T.z_mask, T.coeff);
        break;
      }
      default:
        throw Failure{QOC_ERR_INVALID_ARG, "unknown term kind"};
    }
  }
  std::vector<PauliString> out;
  for (auto& kv : acc)
    if (kv.second != 0.0) out.push_back(PauliString{kv.first.first, kv.first.second, kv.second});
  return out;
}

// Exact invariance: the map string -> coefficient is unchanged by each generator.
static void check_invariant(const std::vector<PauliString>& ps, int n, int s, bool refl, const char* what) {
  std::map<std::pair<uint64_t, uint64_t>, double> ref;
  for (auto& p : ps) ref[{p.x, p.z}] = p.coeff;
  for (int gen = 0; gen < (refl ? 2 : 1); ++gen) {
    for (auto& p : ps) {
      uint64_t gx = gen == 0 ? rotl_n(p.x, s, n) : reflect_n(p.x, n);
      uint64_t gz = gen == 0 ? rotl_n(p.z, s, n) : reflect_n(p.z, n);
      auto it = ref.find({gx, gz});
      QOC_REQUIRE(it != ref.end() && it->second == p.coeff, QOC_ERR_SYMMETRY,
                  std::string(what) + " is not invariant under the " + (gen == 0 ? "rotation" : "reflection"));
    }
  }
}

// ------------------------------------------------------------------- device projection
struct ProjBlock {
  int32_t kind, chi_rho, chi_phi, mom, m, mp;
  int64_t rep_off;
  int64_t h_off;
};

__global__ void k_project(ProjBlock B, const uint64_t* reps_all, const int32_t* per_all, int n, int s, int L,
                          int refl, const PauliString* strings, const int32_t* op_begin, int nops, double* H) {
  int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= B.m) return;
  const uint64_t* reps = reps_all + B.rep_off;
  const int32_t* per = per_all + B.rep_off;
  const uint64_t a = reps[col];
  const double Oa = (double)per[col];
  const bool mom = B.kind != IRR_1D;
  const double twopi = 6.283185307179586476925286766559;
  const size_t plane = (size_t)B.mp * B.mp;
  for (int o = 0; o < nops; ++o) {
    double* Hre = H + B.h_off + (size_t)(2 * o) * plane;
    double* Him = Hre + plane;
    for (int t = op_begin[o]; t < op_begin[o + 1]; ++t) {
      const PauliString P = strings[t];
      const uint64_t x = a ^ P.x;
      // i^{popc(x&z)} * (-1)^{popc(a&z)} as a quarter-turn count
      const int q = (popc64(P.x & P.z) + 2 * popc64(a & P.z)) & 3;
      Canon c = canonicalize(x, n, s, L, mom ? false : (refl != 0));
      // binary search of the representative among the block's columns
      int lo = 0, hi = B.m - 1, row = -1;
      while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        uint64_t v = reps[mid];
        if (v == c.rep) { row = mid; break; }
        if (v < c.rep) lo = mid + 1; else hi = mid - 1;
      }
      if (row < 0) continue;  // representative not allowed by the irrep: contributions cancel
      double re = 0.0, im = 0.0;
      // value = coeff * i^q
      const double cf = P.coeff;
      if (q == 0) re = cf; else if (q == 1) im = cf; else if (q == 2) re = -cf; else im = -cf;
      double fac = sqrt(Oa / (double)per[row]);
      if (!mom) {
        // chi(g_x) with g_x the inverse of rho^l phi^f; real characters are their own inverse
        double chi = (((c.l & 1) && B.chi_rho < 0) ? -1.0 : 1.0) * ((c.f && B.chi_phi < 0) ? -1.0 : 1.0);
        fac *= chi;
        re *= fac;
        im *= fac;
      } else {
        // g_x = rho^{-l}: chi_k(g_x) = exp(-i k l)
        double ang = -twopi * (double)(((int64_t)B.mom * c.l) % L) / (double)L;
        double cr = cos(ang) * fac, ci = sin(ang) * fac;
        double r2 = re * cr - im * ci, i2 = re * ci + im * cr;
        re = r2;
        im = i2;
      }
      size_t idx = (size_t)row + (size_t)col * B.mp;
      Hre[idx] += re;
      Him[idx] += im;
    }
  }
}

__global__ void k_to_float(const double* in, float* out, int64_t count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = (float)in[i];
}

// column sums of |h| for one operator block (FP64); thread per column
__global__ void k_colsum_abs(const double* Hre, const double* Him, int m, int mp, double* out) {
  int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= m) return;
  double s = 0.0;
  for (int r = 0; r < m; ++r) {
    size_t i = (size_t)r + (size_t)col * mp;
    s += hypot(Hre[i], Him[i]);
  }
  out[col] = s;
}

__global__ void k_interleave(const double* re, const double* im, int m, int mp, double2* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)m * m) return;
  int r = (int)(i % m), c = (int)(i / m);
  size_t s = (size_t)r + (size_t)c * mp;
  out[i] = make_double2(re[s], im[s]);
}

// ------------------------------------------------------------------- S_n closed form
// |J,M>, M = J..-J: 2S_z = diag(2M); S_+|J,M> = sqrt(J(J+1) - M(M+1)) |J,M+1>;
// sum_q sigma_a^(q) = 2 S_a and sum_{q<q'} sigma_a^(q) sigma_a^(q') = ((2 S_a)^2 - n) / 2.
static std::vector<std::complex<double>> sn_matrix(int n, int twoJ, const qoc_term* terms, int count) {
  const int d = twoJ + 1;
  using C = std::complex<double>;
  std::vector<C> Sx(d * d), Sy(d * d), Sz(d * d), H(d * d, 0.0);
  const double J = twoJ / 2.0;
  for (int r = 0; r < d; ++r) {
    double M = J - r;
    Sz[r + r * d] = 2.0 * M;
    if (r >= 1) {
      double v = std::sqrt(J * (J + 1) - M * (M + 1));  // <M+1| S_+ |M>, M+1 at row r-1
      // 2S_x = S_+ + S_-, 2S_y = -i (S_+ - S_-)
      Sx[(r - 1) + r * d] += v;
      Sx[r + (r - 1) * d] += v;
      Sy[(r - 1) + r * d] += C(0, -v);
      Sy[r + (r - 1) * d] += C(0, v);
    }
  }
  auto pick = [&](char a) -> std::vector<C>& {
    if (a == 'x' || a == 'X') return Sx;
    if (a == 'y' || a == 'Y') return Sy;
    return Sz;
  };
  for (int t = 0; t < count; ++t) {
    const qoc_term& T = terms[t];
    QOC_REQUIRE(std::isfinite(T.coeff), QOC_ERR_INVALID_ARG, "non-finite term coefficient");
    auto valid = [](char a) { return a == 'x' || a == 'y' || a == 'z' || a == 'X' || a == 'Y' || a == 'Z'; };
    if (T.kind == QOC_TERM_ONE_BODY) {
      QOC_REQUIRE(valid(T.op_a), QOC_ERR_INVALID_ARG, "bad Pauli letter");
      QOC_REQUIRE(T.sites == QOC_SITES_ALL && !T.staggered, QOC_ERR_SYMMETRY,
                  "one-body term with site selection or staggering breaks S_n");
      auto& S = pick(T.op_a);
      for (int i = 0; i < d * d; ++i) H[i] += T.coeff * S[i];
    } else if (T.kind == QOC_TERM_ALL_PAIRS) {
      QOC_REQUIRE(valid(T.op_a) && valid(T.op_b), QOC_ERR_INVALID_ARG, "bad Pauli letter");
      QOC_REQUIRE(std::tolower(T.op_a) == std::tolower(T.op_b), QOC_ERR_SYMMETRY,
                  "mixed all-pairs term is not S_n symmetric");
      auto& S = pick(T.op_a);
      for (int c = 0; c < d; ++c)
        for (int r = 0; r < d; ++r) {
          C acc = 0.0;
          for (int k = 0; k < d; ++k) acc += S[r + k * d] * S[k + c * d];
          if (r == c) acc -= (double)n;
          H[r + c * d] += T.coeff * acc * 0.5;
        }
    } else {
      throw Failure{QOC_ERR_SYMMETRY, "only uniform one-body and all-pairs terms are S_n symmetric"};
    }
  }
  return H;
}

}  // namespace qoc

using namespace qoc;

extern "C" {

qoc_status qoc_project(qoc_basis B, const qoc_term* h0, int n_h0, const qoc_term* hk, const int* n_hk, int K,
                       void* stream, qoc_system* out) {
  return guarded([&] {
    QOC_REQUIRE(B && out, QOC_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    QOC_REQUIRE(K >= 0 && K <= kMaxControls, QOC_ERR_INVALID_ARG, "K must be in 0..32");
    QOC_REQUIRE(n_h0 >= 0 && (n_h0 == 0 || h0), QOC_ERR_INVALID_ARG, "bad H0 term list");
    QOC_REQUIRE(K == 0 || n_hk, QOC_ERR_INVALID_ARG, "n_hk is null");
    int total_hk = 0;
    for (int k = 0; k < K; ++k) {
      QOC_REQUIRE(n_hk[k] >= 0, QOC_ERR_INVALID_ARG, "negative term count");
      total_hk += n_hk[k];
    }
    QOC_REQUIRE(total_hk == 0 || hk, QOC_ERR_INVALID_ARG, "hk is null");
    hipStream_t st = (hipStream_t)stream;
    auto S = std::make_unique<qoc_system_s>();
    S->basis = B;
    S->K = K;
    const int nops = K + 1;
    int64_t elems = 0;
    for (auto& bi : B->blocks) {
      qoc_system_s::Block blk{};
      blk.m = bi.m;
      blk.mp = pad_dim(bi.m);
      blk.d = bi.d;
      blk.h_off = elems;
      blk.state_off = bi.state_off;
      blk.index = (int)S->blocks.size();
      elems += (int64_t)2 * nops * blk.mp * blk.mp;
      S->blocks.push_back(blk);
    }
    S->h_elems = elems;
    auto op_terms = [&](int o, const qoc_term** tl, int* cnt) {
      *tl = o == 0 ? h0 : hk;
      *cnt = o == 0 ? n_h0 : n_hk[o - 1];
      if (o > 0)
        for (int k = 0; k < o - 1; ++k) *tl += n_hk[k];
    };
    // every term is expanded and checked on the host before any device work
    std::vector<PauliString> all;
    std::vector<int32_t> op_begin{0};
    std::vector<double> host;
    if (B->group == QOC_GROUP_SYMMETRIC) {
      host.assign(elems, 0.0);
      for (size_t b = 0; b < B->blocks.size(); ++b) {
        auto& blk = S->blocks[b];
        const size_t plane = (size_t)blk.mp * blk.mp;
        for (int o = 0; o < nops; ++o) {
          const qoc_term* tl;
          int cnt;
          op_terms(o, &tl, &cnt);
          auto M = sn_matrix(B->n, B->blocks[b].twoJ, tl, cnt);
          double* re = host.data() + blk.h_off + (size_t)(2 * o) * plane;
          double* im = re + plane;
          double nrm = 0.0;
          for (int c = 0; c < blk.m; ++c) {
            double cs = 0.0;
            for (int r = 0; r < blk.m; ++r) {
              re[r + (size_t)c * blk.mp] = M[r + c * blk.m].real();
              im[r + (size_t)c * blk.mp] = M[r + c * blk.m].imag();
              cs += std::abs(M[r + c * blk.m]);
            }
            nrm = std::max(nrm, cs);
          }
          blk.norm1.push_back(nrm);
        }
      }
    } else {
      for (int o = 0; o < nops; ++o) {
        const qoc_term* tl;
        int cnt;
        op_terms(o, &tl, &cnt);
        auto ps = expand_terms(B->n, tl, cnt);
        std::string what = o == 0 ? "H0" : "H_" + std::to_string(o);
        check_invariant(ps, B->n, B->stride, B->reflection, what.c_str());
        all.insert(all.end(), ps.begin(), ps.end());
        op_begin.push_back((int32_t)all.size());
      }
    }
    S->h64.alloc(elems * sizeof(double));
    S->h32.alloc(elems * sizeof(float));
    if (B->group == QOC_GROUP_SYMMETRIC) {
      QOC_HIP(hipMemcpyAsync(S->h64.ptr, host.data(), elems * sizeof(double), hipMemcpyHostToDevice, st));
      QOC_HIP(hipStreamSynchronize(st));
    } else {
      QOC_HIP(hipMemsetAsync(S->h64.ptr, 0, elems * sizeof(double), st));
      DeviceBuffer dstr(std::max<size_t>(1, all.size()) * sizeof(PauliString));
      DeviceBuffer dbeg(op_begin.size() * sizeof(int32_t));
      QOC_HIP(hipMemcpyAsync(dstr.ptr, all.data(), all.size() * sizeof(PauliString), hipMemcpyHostToDevice, st));
      QOC_HIP(hipMemcpyAsync(dbeg.ptr, op_begin.data(), op_begin.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
      for (size_t b = 0; b < B->blocks.size(); ++b) {
        const auto& bi = B->blocks[b];
        const auto& blk = S->blocks[b];
        ProjBlock pb{bi.kind, bi.chi_rho, bi.chi_phi, bi.mom, bi.m, blk.mp, bi.rep_off, blk.h_off};
        hipLaunchKernelGGL(k_project, dim3((bi.m + 127) / 128), dim3(128), 0, st, pb, B->d_block_reps.as<uint64_t>(),
                           B->d_block_per.as<int32_t>(), B->n, B->stride, B->L, B->reflection ? 1 : 0,
                           dstr.as<PauliString>(), dbeg.as<int32_t>(), nops, S->h64.as<double>());
        QOC_HIP(hipGetLastError());
      }
      // exact 1-norms of every operator block (FP64), reduced on the host
      for (size_t b = 0; b < B->blocks.size(); ++b) {
        auto& blk = S->blocks[b];
        const size_t plane = (size_t)blk.mp * blk.mp;
        DeviceBuffer cs(blk.m * sizeof(double));
        std::vector<double> h(blk.m);
        for (int o = 0; o < nops; ++o) {
          const double* re = S->h64.as<double>() + blk.h_off + (size_t)(2 * o) * plane;
          hipLaunchKernelGGL(k_colsum_abs, dim3((blk.m + 127) / 128), dim3(128), 0, st, re, re + plane, blk.m, blk.mp,
                             cs.as<double>());
          QOC_HIP(hipGetLastError());
          QOC_HIP(hipMemcpyAsync(h.data(), cs.ptr, blk.m * sizeof(double), hipMemcpyDeviceToHost, st));
          QOC_HIP(hipStreamSynchronize(st));
          blk.norm1.push_back(*std::max_element(h.begin(), h.end()));
        }
      }
    }
    hipLaunchKernelGGL(k_to_float, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0, st, S->h64.as<double>(),
                       S->h32.as<float>(), elems);
    QOC_HIP(hipGetLastError());
    QOC_HIP(hipStreamSynchronize(st));
    *out = S.release();
  });
}

void qoc_system_free(qoc_system s) { delete s; }

qoc_status qoc_check_symmetry(int n, int group, int stride, const qoc_term* terms, int count) {
  return guarded([&] {
    QOC_REQUIRE(count >= 0 && (count == 0 || terms), QOC_ERR_INVALID_ARG, "null term array");
    if (group == QOC_GROUP_SYMMETRIC) {
      QOC_REQUIRE(n >= 1 && n <= 4096, QOC_ERR_INVALID_ARG, "n must be in 1..4096 for the symmetric group");
      (void)sn_matrix(n, n % 2, terms, count);  // validates the term kinds
      return;
    }
    QOC_REQUIRE(group == QOC_GROUP_DIHEDRAL || group == QOC_GROUP_CYCLIC, QOC_ERR_INVALID_ARG, "unknown group");
    QOC_REQUIRE(n >= 1 && n <= 64, QOC_ERR_INVALID_ARG, "n must be in 1..64");
    QOC_REQUIRE(stride >= 1 && stride <= n && n % stride == 0, QOC_ERR_INVALID_ARG, "stride must divide n");
    auto ps = expand_terms(n, terms, count);
    check_invariant(ps, n, stride, group == QOC_GROUP_DIHEDRAL, "operator");
  });
}

qoc_status qoc_system_block(qoc_system S, int block, int op, void* dst_dev, void* stream) {
  return guarded([&] {
    QOC_REQUIRE(S && dst_dev, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(block >= 0 && block < (int)S->blocks.size(), QOC_ERR_INVALID_ARG, "block index out of range");
    QOC_REQUIRE(op >= 0 && op <= S->K, QOC_ERR_INVALID_ARG, "operator index out of range");
    const auto& blk = S->blocks[block];
    const size_t plane = (size_t)blk.mp * blk.mp;
    const double* re = S->h64.as<double>() + blk.h_off + (size_t)(2 * op) * plane;
    int64_t cnt = (int64_t)blk.m * blk.m;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_interleave, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, re, re + plane, blk.m,
                       blk.mp, (double2*)dst_dev);
    QOC_HIP(hipGetLastError());
    QOC_HIP(hipStreamSynchronize(st));
  });
}

}  // extern "C"
