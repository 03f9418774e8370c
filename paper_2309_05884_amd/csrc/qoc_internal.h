// Internal declarations of the gfx950 GRAPE library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/qoc.h"

namespace qoc {

// control operators per system (per-qubit x and y fields of up to 16 qubits)
constexpr int kMaxControls = 32;
// systems with at most this many controls get the generator's operator products (the
// products grow as K^3: 50 per block at K = 4)
constexpr int kMaxPowK = 4;
__host__ __device__ inline int pair_count(int K) { return (K + 1) * (K + 2) / 2; }
__host__ __device__ inline int triple_count(int K) { return (K + 1) * (K + 2) * (K + 3) / 6; }

// ---------------------------------------------------------------------------------------
// error plumbing
void set_error(const std::string& msg);
void clear_error();

struct Failure {
  qoc_status status;
  std::string msg;
};

#define QOC_REQUIRE(cond, code, msg)                      \
  do {                                                    \
    if (!(cond)) throw ::qoc::Failure{(code), (msg)};     \
  } while (0)

#define QOC_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::qoc::Failure{QOC_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

template <class F>
qoc_status guarded(F&& f) {
  try {
    clear_error();
    f();
    return QOC_OK;
  } catch (const Failure& e) {
    set_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return QOC_ERR_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    set_error(e.what());
    return QOC_ERR_INVALID_ARG;
  }
}

// ---------------------------------------------------------------------------------------
// device buffers owned by handles (set-up only; never on the hot path)
struct DeviceBuffer {
  void* ptr = nullptr;
  size_t bytes = 0;
  DeviceBuffer() = default;
  explicit DeviceBuffer(size_t n) { alloc(n); }
  DeviceBuffer(const DeviceBuffer&) = delete;
  DeviceBuffer& operator=(const DeviceBuffer&) = delete;
  DeviceBuffer(DeviceBuffer&& o) noexcept : ptr(o.ptr), bytes(o.bytes) { o.ptr = nullptr; o.bytes = 0; }
  DeviceBuffer& operator=(DeviceBuffer&& o) noexcept {
    release();
    ptr = o.ptr; bytes = o.bytes; o.ptr = nullptr; o.bytes = 0;
    return *this;
  }
  ~DeviceBuffer() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) n = 256;
    hipError_t e = hipMalloc(&ptr, n);
    if (e != hipSuccess) {
      ptr = nullptr;
      throw Failure{QOC_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e)};
    }
    bytes = n;
  }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(ptr); }
};

// ---------------------------------------------------------------------------------------
// Pauli strings over bit positions: operator = coeff * i^{popc(x&z)} X^x Z^z, so that
// P|a> = coeff * i^{popc(x&z)} (-1)^{popc(a&z)} |a ^ x>.
struct PauliString {
  uint64_t x;
  uint64_t z;
  double coeff;
};

// ---------------------------------------------------------------------------------------
// group/basis data
enum IrrepKind : int32_t { IRR_1D = 0, IRR_E = 1, IRR_MOMENTUM = 2, IRR_SPIN = 3 };

struct BlockInfo {
  std::string label;
  int32_t kind;      // IrrepKind
  int32_t chi_rho;   // 1-dim irreps: character of rho (+1/-1)
  int32_t chi_phi;   // 1-dim irreps: character of phi (+1/-1)
  int32_t mom;       // E_m / k_m: momentum index m
  int32_t m;         // block size
  int32_t d;         // copies
  int32_t twoJ;      // spin blocks
  int64_t rep_off;   // offset of the block's representatives in basis rep storage
  int64_t state_off; // offset of the block in a state panel (complex entries)
};

}  // namespace qoc

struct qoc_basis_s {
  int n = 0;
  int group = 0;
  int stride = 1;
  int L = 1;
  bool reflection = false;
  std::vector<qoc::BlockInfo> blocks;
  int64_t dim = 0;                       // panel length D
  std::vector<uint64_t> h_greps, h_creps;  // orbit representatives (group / rotations)
  std::vector<uint64_t> h_block_reps;    // concatenated block representatives
  std::vector<int32_t> h_block_per;      // orbit size (1-dim) or period (E) per block rep
  qoc::DeviceBuffer d_block_reps;        // uint64
  qoc::DeviceBuffer d_block_per;         // int32
};

struct qoc_system_s {
  qoc_basis_s* basis = nullptr;  // borrowed: the basis must outlive the system
  int K = 0;
  struct Block {
    int m, mp, d;
    int index;            // position in the system's block list
    int64_t h_off;        // element offset of the block's operator planes
    int64_t state_off;    // complex offset in state panels
    std::vector<double> norm1;  // exact 1-norm of each operator block (host)
  };
  std::vector<Block> blocks;
  // Operator planes: for block b, operator o (0 = H0), plane c (0 re, 1 im):
  //   base + h_off + ((size_t)(2*o + c)) * mp*mp, column-major mp x mp, zero padded.
  qoc::DeviceBuffer h64;  // double
  qoc::DeviceBuffer h32;  // float
  int64_t h_elems = 0;
  // Symmetrised operator products from which the generator forms the second and third
  // powers of a slice's exponent by linear combination (formed once, when a plan first
  // needs them, for K <= kMaxPowK): per block, the pair products S_ab = H_a H_b + H_b H_a
  // (a < b) and S_aa = H_a^2, (K+1)(K+2)/2 of them with (a, b) in lexicographic order, then
  // the triple products T_abc = sum of H_x H_y H_z over the distinct orderings (x, y, z) of
  // (a, b, c), a <= b <= c, (K+1)(K+2)(K+3)/6 of them; planes as the operators' (re, im;
  // column-major mp x mp, zero padded), FP64 and / or FP32 (whichever plans have needed).
  qoc::DeviceBuffer pw64, pw32;
  std::vector<int64_t> pw_off;  // element offset of each block's products
};

namespace qoc {
constexpr int kPad = 16;        // matrix dimensions are padded to a multiple of the MFMA tile
inline int pad_dim(int m) { return (m + kPad - 1) / kPad * kPad; }

// hot-path entry implemented in grape.hip
struct Plan;
}  // namespace qoc
