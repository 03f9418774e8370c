// Orbit enumeration, symmetry-adapted block tables and dense <-> block state maps
// (Sec. II A, Table I; App. A, Eqs. (A1)-(A2)).
//
// Every basis state x of the 2^n register is canonicalised on the device to the
// minimum of its orbit (rotations, and for the dihedral group reflections, of the bit
// string).  Representatives are stream-compacted in ascending order, their stabiliser
// data computed, and each irrep's block keeps the representatives whose stabiliser the
// irrep's character is trivial on (momentum blocks: m * period = 0 mod L).  The host
// cross-checks every block size against the character formula.
#include <algorithm>
#include <cmath>
#include <complex>
#include <mutex>
#include <numeric>

#include "bits.h"
#include "qoc_internal.h"

namespace qoc {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

// ------------------------------------------------------------------------------- kernels
// flags bit 0: x is the minimum of its orbit under the whole group
// flags bit 1: x is the minimum of its orbit under the rotations only
__global__ void k_orbit_flags(int n, int s, int L, int refl, uint64_t count, uint8_t* flags) {
  uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= count) return;
  Canon g = canonicalize(x, n, s, L, refl != 0);
  Canon c = canonicalize(x, n, s, L, false);
  flags[x] = (uint8_t)((g.rep == x ? 1 : 0) | (c.rep == x ? 2 : 0));
}

// Predicate for compaction.
struct Pred {
  int mode;        // 0: flags[i] & bit over implicit i; 1: attr[i] & bit; 2: (m * per[i]) % L == 0
  int bit;
  int m;
  int L;
  const uint8_t* flags;
  const uint32_t* attr;
  const int32_t* per;
  const uint64_t* vals;  // mode 1/2: values to compact (implicit index i for mode 0)
  const int32_t* vals_per;  // optional companion array compacted alongside (mode 1/2)
  __device__ bool test(uint64_t i) const {
    if (mode == 0) return (flags[i] & bit) != 0;
    if (mode == 1) return (attr[i] & (uint32_t)bit) != 0;
    return ((int64_t)m * per[i]) % L == 0;
  }
  __device__ uint64_t value(uint64_t i) const { return mode == 0 ? i : vals[i]; }
};

constexpr int kChunk = 256;

__device__ inline int wg_exclusive_scan(int v, int* lds, int* total) {
  // 256 threads = 4 waves of 64
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    int t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) lds[wave] = incl;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wave; ++w) base += lds[w];
  *total = lds[0] + lds[1] + lds[2] + lds[3];
  __syncthreads();
  return base + incl - v;
}

__global__ void k_compact_count(Pred p, uint64_t count, uint32_t* chunk_counts) {
  __shared__ int lds[4];
  uint64_t i = (uint64_t)blockIdx.x * kChunk + threadIdx.x;
  int v = (i < count && p.test(i)) ? 1 : 0;
  int total;
  (void)wg_exclusive_scan(v, lds, &total);
  if (threadIdx.x == 0) chunk_counts[blockIdx.x] = (uint32_t)total;
}

// single work-group exclusive scan of chunk counts (64-bit offsets), total at offs[nchunks]
__global__ void k_compact_scan(const uint32_t* counts, uint64_t nchunks, uint64_t* offs) {
  __shared__ int lds[4];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint64_t base = 0; base < nchunks; base += kChunk) {
    uint64_t i = base + threadIdx.x;
    int v = i < nchunks ? (int)counts[i] : 0;
    int total;
    int ex = wg_exclusive_scan(v, lds, &total);
    if (i < nchunks) offs[i] = carry + (uint64_t)ex;
    __syncthreads();
    if (threadIdx.x == 0) carry += (uint64_t)total;
    __syncthreads();
  }
  if (threadIdx.x == 0) offs[nchunks] = carry;
}

__global__ void k_compact_scatter(Pred p, uint64_t count, const uint64_t* offs, uint64_t* out,
                                  int32_t* out_per) {
  __shared__ int lds[4];
  uint64_t i = (uint64_t)blockIdx.x * kChunk + threadIdx.x;
  int v = (i < count && p.test(i)) ? 1 : 0;
  int total;
  int ex = wg_exclusive_scan(v, lds, &total);
  if (v) {
    uint64_t o = offs[blockIdx.x] + (uint64_t)ex;
    out[o] = p.value(i);
    if (out_per) out_per[o] = p.vals_per[i];
  }
}

// Stabiliser data of group representatives: orbit size, and bit c set when the
// one-dimensional irrep c (0 A1, 1 A2, 2 B1, 3 B2) is trivial on the stabiliser.
__global__ void k_group_rep_attrs(const uint64_t* reps, uint64_t count, int n, int s, int L, int refl,
                                  int32_t* orbit, uint32_t* compat) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint64_t a = reps[i];
  int stab = 0;
  int ok[4] = {1, 1, 1, 1};
  const int crho[4] = {1, 1, -1, -1};
  const int cphi[4] = {1, -1, 1, -1};
  for (int f = 0; f <= (refl ? 1 : 0); ++f) {
    for (int l = 0; l < L; ++l) {
      if (group_act(a, l, f, n, s) == a) {
        ++stab;
        for (int c = 0; c < 4; ++c) {
          int chi = ((l & 1) && crho[c] < 0 ? -1 : 1) * (f && cphi[c] < 0 ? -1 : 1);
          if (chi != 1) ok[c] = 0;
        }
      }
    }
  }
  int order = refl ? 2 * L : L;
  orbit[i] = order / stab;
  compat[i] = (uint32_t)(ok[0] | (ok[1] << 1) | (ok[2] << 2) | (ok[3] << 3));
}

// Rotation period of cyclic representatives.
__global__ void k_cyclic_period(const uint64_t* reps, uint64_t count, int n, int s, int L, int32_t* per) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint64_t c = reps[i];
  uint64_t y = c;
  int P = L;
  for (int l = 1; l <= L; ++l) {
    y = rotl_n(y, s, n);
    if (y == c) { P = l; break; }
  }
  per[i] = P;
}

// ------------------------------------------------------------------------- host helpers
static void compact(const Pred& p, uint64_t count, DeviceBuffer& out_vals, DeviceBuffer* out_per,
                    uint64_t* out_count, hipStream_t st) {
  uint64_t nchunks = (count + kChunk - 1) / kChunk;
  DeviceBuffer counts(std::max<uint64_t>(1, nchunks) * sizeof(uint32_t));
  DeviceBuffer offs((nchunks + 1) * sizeof(uint64_t));
  if (nchunks) {
    hipLaunchKernelGGL(k_compact_count, dim3((unsigned)nchunks), dim3(kChunk), 0, st, p, count,
                       counts.as<uint32_t>());
    QOC_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(kChunk), 0, st, counts.as<uint32_t>(), nchunks,
                     offs.as<uint64_t>());
  QOC_HIP(hipGetLastError());
  uint64_t total = 0;
  QOC_HIP(hipMemcpyAsync(&total, offs.as<uint64_t>() + nchunks, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
  QOC_HIP(hipStreamSynchronize(st));
  out_vals.alloc(std::max<uint64_t>(1, total) * sizeof(uint64_t));
  if (out_per) out_per->alloc(std::max<uint64_t>(1, total) * sizeof(int32_t));
  if (nchunks) {
    hipLaunchKernelGGL(k_compact_scatter, dim3((unsigned)nchunks), dim3(kChunk), 0, st, p, count,
                       offs.as<uint64_t>(), out_vals.as<uint64_t>(), out_per ? out_per->as<int32_t>() : nullptr);
    QOC_HIP(hipGetLastError());
  }
  QOC_HIP(hipStreamSynchronize(st));  // scratch buffers are released on return
  *out_count = total;
}

static int perm_cycles(int n, int s, int l, int f) {
  std::vector<int> seen(n, 0);
  int c = 0;
  for (int p = 0; p < n; ++p) {
    if (seen[p]) continue;
    ++c;
    int q = p;
    while (!seen[q]) {
      seen[q] = 1;
      int img = f ? (-q + l * s) : (q + l * s);
      q = ((img % n) + n) % n;
    }
  }
  return c;
}

// Multiplicity of an irrep in the permutation representation, from its characters.
static long long character_size(const BlockInfo& b, int n, int s, int L, bool refl) {
  const double pi = 3.14159265358979323846;
  std::complex<double> tot = 0.0;
  for (int f = 0; f <= (refl ? 1 : 0); ++f) {
    for (int l = 0; l < L; ++l) {
      std::complex<double> chi;
      if (b.kind == IRR_1D) {
        chi = ((l & 1) && b.chi_rho < 0 ? -1.0 : 1.0) * (f && b.chi_phi < 0 ? -1.0 : 1.0);
      } else if (b.kind == IRR_E) {
        chi = f ? 0.0 : 2.0 * std::cos(2 * pi * b.mom * l / L);
      } else {
        chi = std::polar(1.0, 2 * pi * b.mom * l / L);
      }
      tot += std::conj(chi) * std::ldexp(1.0, perm_cycles(n, s, l, f));
    }
  }
  tot /= (double)(refl ? 2 * L : L);
  return std::llround(tot.real());
}

static std::vector<BlockInfo> ring_irreps(int L, bool refl) {
  std::vector<BlockInfo> v;
  auto mk = [](const char* lab, int kind, int cr, int cp, int mom) {
    BlockInfo b{};
    b.label = lab;
    b.kind = kind;
    b.chi_rho = cr;
    b.chi_phi = cp;
    b.mom = mom;
    b.d = kind == IRR_E ? 2 : 1;
    return b;
  };
  if (refl) {
    v.push_back(mk("A1", IRR_1D, 1, 1, 0));
    v.push_back(mk("A2", IRR_1D, 1, -1, 0));
    if (L % 2 == 0) {
      v.push_back(mk("B1", IRR_1D, -1, 1, 0));
      v.push_back(mk("B2", IRR_1D, -1, -1, 0));
    }
    int nE = (L % 2) ? (L - 1) / 2 : L / 2 - 1;
    for (int m = 1; m <= nE; ++m) {
      BlockInfo b = mk("E", IRR_E, 0, 0, m);
      b.label = "E" + std::to_string(m);
      v.push_back(b);
    }
  } else {
    for (int m = 0; m < L; ++m) {
      BlockInfo b = mk("k", IRR_MOMENTUM, 0, 0, m);
      b.label = "k" + std::to_string(m);
      v.push_back(b);
    }
  }
  return v;
}

static void build_ring_basis(qoc_basis_s* B, hipStream_t st) {
  const int n = B->n, s = B->stride, L = B->L;
  const bool refl = B->reflection;
  const uint64_t count = 1ull << n;
  DeviceBuffer flags(count);
  hipLaunchKernelGGL(k_orbit_flags, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, n, s, L,
                     refl ? 1 : 0, count, flags.as<uint8_t>());
  QOC_HIP(hipGetLastError());

  Pred pg{};
  pg.mode = 0;
  pg.bit = 1;
  pg.flags = flags.as<uint8_t>();
  Pred pc = pg;
  pc.bit = 2;
  DeviceBuffer greps, creps;
  uint64_t ng = 0, nc = 0;
  compact(pg, count, greps, nullptr, &ng, st);
  compact(pc, count, creps, nullptr, &nc, st);

  DeviceBuffer gorb(std::max<uint64_t>(1, ng) * 4), gcompat(std::max<uint64_t>(1, ng) * 4);
  DeviceBuffer cper(std::max<uint64_t>(1, nc) * 4);
  if (ng)
    hipLaunchKernelGGL(k_group_rep_attrs, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, st, greps.as<uint64_t>(),
                       ng, n, s, L, refl ? 1 : 0, gorb.as<int32_t>(), gcompat.as<uint32_t>());
  if (nc)
    hipLaunchKernelGGL(k_cyclic_period, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, creps.as<uint64_t>(),
                       nc, n, s, L, cper.as<int32_t>());
  QOC_HIP(hipGetLastError());

  B->h_greps.resize(ng);
  B->h_creps.resize(nc);
  QOC_HIP(hipMemcpyAsync(B->h_greps.data(), greps.ptr, ng * 8, hipMemcpyDeviceToHost, st));
  QOC_HIP(hipMemcpyAsync(B->h_creps.data(), creps.ptr, nc * 8, hipMemcpyDeviceToHost, st));

  std::vector<BlockInfo> irr = ring_irreps(L, refl);
  std::vector<DeviceBuffer> bl_reps(irr.size()), bl_per(irr.size());
  std::vector<uint64_t> bl_count(irr.size(), 0);
  int c1 = 0;
  for (size_t b = 0; b < irr.size(); ++b) {
    Pred p{};
    if (irr[b].kind == IRR_1D) {
      p.mode = 1;
      p.bit = 1 << c1++;
      p.attr = gcompat.as<uint32_t>();
      p.vals = greps.as<uint64_t>();
      p.vals_per = gorb.as<int32_t>();
      compact(p, ng, bl_reps[b], &bl_per[b], &bl_count[b], st);
    } else {
      p.mode = 2;
      p.m = irr[b].mom;
      p.L = L;
      p.per = cper.as<int32_t>();
      p.vals = creps.as<uint64_t>();
      p.vals_per = cper.as<int32_t>();
      compact(p, nc, bl_reps[b], &bl_per[b], &bl_count[b], st);
    }
  }
  QOC_HIP(hipStreamSynchronize(st));

  // host copies, block offsets and the character cross-check
  int64_t rep_off = 0, state_off = 0;
  B->blocks.clear();
  for (size_t b = 0; b < irr.size(); ++b) {
    BlockInfo bi = irr[b];
    bi.m = (int32_t)bl_count[b];
    long long expect = character_size(bi, n, s, L, refl);
    QOC_REQUIRE(expect == bi.m, QOC_ERR_NUMERIC,
                "block " + bi.label + ": enumerated size " + std::to_string(bi.m) +
                    " differs from the character formula " + std::to_string(expect));
    bi.rep_off = rep_off;
    bi.state_off = state_off;
    rep_off += bi.m;
    state_off += (int64_t)bi.m * bi.d;
    B->blocks.push_back(bi);
  }
  QOC_REQUIRE(state_off == (int64_t)count, QOC_ERR_NUMERIC, "block dimensions do not sum to 2^n");
  B->dim = state_off;
  B->h_block_reps.resize(rep_off);
  B->h_block_per.resize(rep_off);
  for (size_t b = 0; b < irr.size(); ++b) {
    if (!bl_count[b]) continue;
    QOC_HIP(hipMemcpy(B->h_block_reps.data() + B->blocks[b].rep_off, bl_reps[b].ptr, bl_count[b] * 8,
                      hipMemcpyDeviceToHost));
    QOC_HIP(hipMemcpy(B->h_block_per.data() + B->blocks[b].rep_off, bl_per[b].ptr, bl_count[b] * 4,
                      hipMemcpyDeviceToHost));
  }
  B->d_block_reps.alloc(std::max<int64_t>(1, rep_off) * 8);
  B->d_block_per.alloc(std::max<int64_t>(1, rep_off) * 4);
  QOC_HIP(hipMemcpy(B->d_block_reps.ptr, B->h_block_reps.data(), rep_off * 8, hipMemcpyHostToDevice));
  QOC_HIP(hipMemcpy(B->d_block_per.ptr, B->h_block_per.data(), rep_off * 4, hipMemcpyHostToDevice));
  // drop empty blocks from the table (e.g. A2 at n = 4); their offsets are unchanged
  std::vector<BlockInfo> kept;
  for (auto& bi : B->blocks)
    if (bi.m > 0) kept.push_back(bi);
  B->blocks.swap(kept);
}

static void build_symmetric_basis(qoc_basis_s* B) {
  int64_t state_off = 0;
  for (int twoJ = B->n; twoJ >= 0; twoJ -= 2) {
    BlockInfo bi{};
    bi.label = "J" + std::to_string(twoJ) + "/2";
    bi.kind = IRR_SPIN;
    bi.twoJ = twoJ;
    bi.m = twoJ + 1;
    bi.d = 1;
    bi.rep_off = 0;
    bi.state_off = state_off;
    state_off += bi.m;
    B->blocks.push_back(bi);
  }
  B->dim = state_off;
}

// ------------------------------------------------------------------- state conversion
struct BlockDev {
  int32_t kind, chi_rho, chi_phi, mom, m, d;
  int64_t rep_off, state_off;
};

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// amplitude of each block basis state: <a,chi,c|psi> (thread per basis state and copy)
__global__ void k_to_blocks(const BlockDev* blocks, int nblocks, const uint64_t* reps, const int32_t* per, int n,
                            int s, int L, int refl, const double2* dense, double2* out, int64_t total) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  int b = 0;
  while (b + 1 < nblocks && blocks[b + 1].state_off <= t) ++b;
  const BlockDev B = blocks[b];
  int64_t local = t - B.state_off;
  int copy = (int)(local / B.m);
  int idx = (int)(local % B.m);
  uint64_t a = reps[B.rep_off + idx];
  int pa = per[B.rep_off + idx];
  const double twopi = 6.283185307179586476925286766559;
  double2 acc = make_double2(0.0, 0.0);
  if (B.kind == IRR_1D) {
    // sum over all group elements counts each orbit member |Stab| times
    int order = refl ? 2 * L : L;
    double scale = 1.0 / ((double)(order / pa) * sqrt((double)pa));
    for (int f = 0; f <= refl; ++f)
      for (int l = 0; l < L; ++l) {
        double chi = (((l & 1) && B.chi_rho < 0) ? -1.0 : 1.0) * ((f && B.chi_phi < 0) ? -1.0 : 1.0);
        double2 v = dense[group_act(a, l, f, n, s)];
        acc.x += chi * v.x;
        acc.y += chi * v.y;
      }
    acc.x *= scale;
    acc.y *= scale;
  } else {
    double sc = 1.0 / sqrt((double)pa);
    for (int l = 0; l < pa; ++l) {
      uint64_t y = rotl_n(a, l * s, n);
      if (copy == 1) y = reflect_n(y, n);
      double ang = twopi * (double)(((int64_t)B.mom * l) % L) / (double)L;
      double2 e = make_double2(cos(ang), sin(ang));  // conj of exp(-i k l)
      double2 v = cmul(e, dense[y]);
      acc.x += sc * v.x;
      acc.y += sc * v.y;
    }
  }
  out[t] = acc;
}

__device__ inline int find_rep(const uint64_t* reps, int m, uint64_t key) {
  int lo = 0, hi = m - 1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    uint64_t v = reps[mid];
    if (v == key) return mid;
    if (v < key) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

// dense amplitude of x: sum over blocks and copies of amplitude * <x|a,chi,c>
__global__ void k_from_blocks(const BlockDev* blocks, int nblocks, const uint64_t* reps, const int32_t* per, int n,
                              int s, int L, int refl, const double2* in, double2* dense, uint64_t count) {
  uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= count) return;
  Canon g = canonicalize(x, n, s, L, refl != 0);
  Canon c = canonicalize(x, n, s, L, false);
  Canon c2{0, 0, 0};
  if (refl) c2 = canonicalize(reflect_n(x, n), n, s, L, false);
  const double twopi = 6.283185307179586476925286766559;
  double2 acc = make_double2(0.0, 0.0);
  for (int b = 0; b < nblocks; ++b) {
    const BlockDev B = blocks[b];
    const uint64_t* r = reps + B.rep_off;
    if (B.kind == IRR_1D) {
      int i = find_rep(r, B.m, g.rep);
      if (i < 0) continue;
      // rho^l phi^f maps x to the representative; the coefficient of |x> is
      // conj(chi(g_x)) / sqrt(|O|) with g_x the inverse, and chi(g^-1) = chi(g) here
      double chi = (((g.l & 1) && B.chi_rho < 0) ? -1.0 : 1.0) * ((g.f && B.chi_phi < 0) ? -1.0 : 1.0);
      double sc = chi / sqrt((double)per[B.rep_off + i]);
      double2 v = in[B.state_off + i];
      acc.x += sc * v.x;
      acc.y += sc * v.y;
    } else {
      // copy 0: x = rho^{-l'} c with rho^{l'} x = c, coefficient exp(-i k (L - l')) / sqrt(P)
      for (int copy = 0; copy < B.d; ++copy) {
        const Canon& cc = copy == 0 ? c : c2;
        int i = find_rep(r, B.m, cc.rep);
        if (i < 0) continue;
        int P = per[B.rep_off + i];
        int lx = ((L - cc.l) % P + P) % P;  // x (or phi x) = rho^{lx} c
        double ang = -twopi * (double)(((int64_t)B.mom * lx) % L) / (double)L;
        double sc = 1.0 / sqrt((double)P);
        double2 v = in[B.state_off + (int64_t)copy * B.m + i];
        double2 e = make_double2(sc * cos(ang), sc * sin(ang));
        double2 w = cmul(e, v);
        acc.x += w.x;
        acc.y += w.y;
      }
    }
  }
  dense[x] = acc;
}

static std::vector<BlockDev> block_dev_table(const qoc_basis_s* B) {
  std::vector<BlockDev> v;
  for (auto& b : B->blocks) v.push_back(BlockDev{b.kind, b.chi_rho, b.chi_phi, b.mom, b.m, b.d, b.rep_off, b.state_off});
  return v;
}

}  // namespace qoc

using namespace qoc;

extern "C" {

const char* qoc_last_error(void) { return g_last_error.c_str(); }

const char* qoc_status_string(qoc_status s) {
  switch (s) {
    case QOC_OK: return "ok";
    case QOC_ERR_INVALID_ARG: return "invalid argument";
    case QOC_ERR_SYMMETRY: return "term breaks the group symmetry";
    case QOC_ERR_UNSUPPORTED: return "unsupported";
    case QOC_ERR_OUT_OF_MEMORY: return "out of memory";
    case QOC_ERR_DEVICE: return "device error";
    case QOC_ERR_NUMERIC: return "numeric check failed";
  }
  return "unknown status";
}

int qoc_version(void) { return 100; }

qoc_status qoc_build_basis(int n, int group, int stride, void* stream, qoc_basis* out) {
  return guarded([&] {
    QOC_REQUIRE(out != nullptr, QOC_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    QOC_REQUIRE(group == QOC_GROUP_DIHEDRAL || group == QOC_GROUP_CYCLIC || group == QOC_GROUP_SYMMETRIC,
                QOC_ERR_INVALID_ARG, "unknown group");
    auto B = std::make_unique<qoc_basis_s>();
    B->n = n;
    B->group = group;
    if (group == QOC_GROUP_SYMMETRIC) {
      QOC_REQUIRE(n >= 1 && n <= 4096, QOC_ERR_INVALID_ARG, "n must be in 1..4096 for the symmetric group");
      B->stride = 1;
      B->L = 1;
      build_symmetric_basis(B.get());
    } else {
      QOC_REQUIRE(n >= 1 && n <= 30, QOC_ERR_INVALID_ARG, "n must be in 1..30 for ring groups");
      QOC_REQUIRE(stride >= 1 && stride <= n && n % stride == 0, QOC_ERR_INVALID_ARG, "stride must divide n");
      B->stride = stride;
      B->L = n / stride;
      B->reflection = group == QOC_GROUP_DIHEDRAL;
      build_ring_basis(B.get(), (hipStream_t)stream);
    }
    *out = B.release();
  });
}

void qoc_basis_free(qoc_basis b) { delete b; }

qoc_status qoc_basis_blocks(qoc_basis B, int* nblocks, int32_t* sizes, int32_t* copies, int cap) {
  return guarded([&] {
    QOC_REQUIRE(B && nblocks, QOC_ERR_INVALID_ARG, "null argument");
    *nblocks = (int)B->blocks.size();
    for (int i = 0; i < (int)B->blocks.size() && i < cap; ++i) {
      if (sizes) sizes[i] = B->blocks[i].m;
      if (copies) copies[i] = B->blocks[i].d;
    }
  });
}

qoc_status qoc_basis_reps(qoc_basis B, int which, uint64_t* reps, int64_t cap, int64_t* count) {
  return guarded([&] {
    QOC_REQUIRE(B && count, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(B->group != QOC_GROUP_SYMMETRIC, QOC_ERR_UNSUPPORTED, "the symmetric group has no enumeration");
    const uint64_t* src = nullptr;
    int64_t cnt = 0;
    if (which == 0) { src = B->h_greps.data(); cnt = (int64_t)B->h_greps.size(); }
    else if (which == 1) { src = B->h_creps.data(); cnt = (int64_t)B->h_creps.size(); }
    else {
      int b = which - 2;
      QOC_REQUIRE(b >= 0 && b < (int)B->blocks.size(), QOC_ERR_INVALID_ARG, "block index out of range");
      src = B->h_block_reps.data() + B->blocks[b].rep_off;
      cnt = B->blocks[b].m;
    }
    *count = cnt;
    if (reps)
      for (int64_t i = 0; i < cnt && i < cap; ++i) reps[i] = src[i];
  });
}

qoc_status qoc_state_to_blocks(qoc_basis B, const void* dense_dev, void* blocks_dev, void* stream) {
  return guarded([&] {
    QOC_REQUIRE(B && dense_dev && blocks_dev, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(B->group != QOC_GROUP_SYMMETRIC, QOC_ERR_UNSUPPORTED, "no dense map for the symmetric group");
    auto tab = block_dev_table(B);
    DeviceBuffer dt(tab.size() * sizeof(BlockDev));
    hipStream_t st = (hipStream_t)stream;
    QOC_HIP(hipMemcpyAsync(dt.ptr, tab.data(), tab.size() * sizeof(BlockDev), hipMemcpyHostToDevice, st));
    int64_t total = B->dim;
    hipLaunchKernelGGL(k_to_blocks, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, dt.as<BlockDev>(),
                       (int)tab.size(), B->d_block_reps.as<uint64_t>(), B->d_block_per.as<int32_t>(), B->n,
                       B->stride, B->L, B->reflection ? 1 : 0, (const double2*)dense_dev, (double2*)blocks_dev, total);
    QOC_HIP(hipGetLastError());
    QOC_HIP(hipStreamSynchronize(st));
  });
}

qoc_status qoc_state_from_blocks(qoc_basis B, const void* blocks_dev, void* dense_dev, void* stream) {
  return guarded([&] {
    QOC_REQUIRE(B && dense_dev && blocks_dev, QOC_ERR_INVALID_ARG, "null argument");
    QOC_REQUIRE(B->group != QOC_GROUP_SYMMETRIC, QOC_ERR_UNSUPPORTED, "no dense map for the symmetric group");
    auto tab = block_dev_table(B);
    DeviceBuffer dt(tab.size() * sizeof(BlockDev));
    hipStream_t st = (hipStream_t)stream;
    QOC_HIP(hipMemcpyAsync(dt.ptr, tab.data(), tab.size() * sizeof(BlockDev), hipMemcpyHostToDevice, st));
    uint64_t count = 1ull << B->n;
    hipLaunchKernelGGL(k_from_blocks, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, dt.as<BlockDev>(),
                       (int)tab.size(), B->d_block_reps.as<uint64_t>(), B->d_block_per.as<int32_t>(), B->n,
                       B->stride, B->L, B->reflection ? 1 : 0, (const double2*)blocks_dev, (double2*)dense_dev, count);
    QOC_HIP(hipGetLastError());
    QOC_HIP(hipStreamSynchronize(st));
  });
}

}  // extern "C"
