/*
 * qoc.h - C ABI of the symmetry-reduced GRAPE hot path for AMD Instinct MI355X (gfx950).
 *
 * The operations follow Wang, Okyay, Kumar & Wong, "Accelerating Quantum Optimal
 * Control of Multi-Qubit Systems with Symmetry-Based Hamiltonian Transformations"
 * (AVS Quantum Sci. 2023):
 *   - Schroedinger dynamics with a static H0 and controls H_c(t) = sum_k u_k(t) H_k
 *     (Sec. II A, Eqs. (1)-(2); Eq. (6) for the global x/y controls);
 *   - piecewise-constant slice propagators U_j = exp(-i dt (H0 + sum_k u[j,k] H_k))
 *     (Eq. (3));
 *   - the state-transfer objective |<psi_f|psi_N>|^2 (Eq. (4)) and its gradient with
 *     respect to every slice sample (App. B, Eq. (B2), here taken exactly);
 *   - the block diagonalisation of ring-symmetric (D_n) and permutation-symmetric (S_n)
 *     Hamiltonians by group-algebra projections (Sec. II A, Table I; App. A,
 *     Eqs. (A1)-(A2)).
 *
 * Conventions used by every entry point
 * -------------------------------------
 * Qubits q = 1..n; qubit q is bit position p = n - q of a basis index (qubit 1 is the
 * most significant bit, the Kronecker order of Sec. II A).  Bit value 0 is spin up.
 * The group acts on bit positions: rotation rho: p -> p + stride (mod n) and, for the
 * dihedral group, the site-centred reflection phi: p -> -p (mod n).  L = n / stride.
 *
 * Blocks (irreps) are ordered A1, A2, B1, B2 (B only for even L), E_1 .. E_{ceil(L/2)-1}
 * for the dihedral group; k_0 .. k_{L-1} (momentum 2 pi m / L) for the cyclic group;
 * J = n/2, n/2 - 1, ... for the symmetric group.  B1 has character -1 on rho and +1 on
 * phi.  Inside a block the basis states are ordered by ascending orbit representative
 * (the minimum integer of the orbit).  For a one-dimensional irrep chi and
 * representative a (allowed when chi is trivial on the stabiliser of a) the basis
 * state is |a,chi> = |O_a|^{-1/2} sum_{y in O_a} conj(chi(g_y)) |y>, g_y a = y.  For
 * E_m the first copy is the momentum state |c,k> = P_c^{-1/2} sum_{l<P_c}
 * exp(-i k l) |rho^l c>, k = 2 pi m / L, over cyclic representatives c of period P_c
 * with m P_c = 0 mod L, and the second copy is U_phi |c,k>; both copies carry the
 * same block matrix.  The symmetric-group blocks use |J,M>, M = J, J-1, ..., -J.
 *
 * Panels.  A state in block form is the concatenation, in block order, of one
 * column-major m x d panel per block (d = copies: 2 for E_m, 1 otherwise), stored as
 * interleaved complex128 (the layout of a torch.complex128 tensor).  Its length is
 * D = sum_blocks m * d (= 2^n for the ring groups; one copy per J for S_n).
 *
 * Controls u are float64 row-major [N][K] device arrays; gradients are float64
 * [N][K] device arrays.  Outputs of the objective are float64 device arrays.
 *
 * Ownership.  Handles (qoc_basis, qoc_system, qoc_plan) are owned by the library
 * until the matching *_free call.  Every array argument is owned by the caller; the
 * library never frees it.  The hot-path calls (qoc_propagate, qoc_fidelity_grad, for
 * single-problem and batched plans alike) allocate nothing: their scratch memory is the
 * caller's workspace, sized by qoc_plan_workspace_size.
 *
 * Errors.  Every call returns a qoc_status; nothing throws or aborts across the ABI.
 * Argument and symmetry checks happen before any device work.  A device failure
 * returns QOC_ERR_DEVICE; qoc_last_error() then holds the HIP error text.  Calls
 * taking a stream enqueue asynchronously on it unless stated otherwise.
 */
#ifndef QOC_H
#define QOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QOC_OK = 0,
  QOC_ERR_INVALID_ARG = 1,   /* null pointer, size out of range, non-finite input */
  QOC_ERR_SYMMETRY = 2,      /* a term is not invariant under the requested group */
  QOC_ERR_UNSUPPORTED = 3,   /* valid request the library does not implement */
  QOC_ERR_OUT_OF_MEMORY = 4, /* workspace too small, or a setup allocation failed */
  QOC_ERR_DEVICE = 5,        /* HIP runtime error */
  QOC_ERR_NUMERIC = 6        /* a numeric check failed (see qoc_last_error) */
} qoc_status;

typedef enum { QOC_GROUP_DIHEDRAL = 0, QOC_GROUP_CYCLIC = 1, QOC_GROUP_SYMMETRIC = 2 } qoc_group;
typedef enum { QOC_C128 = 0, QOC_C64 = 1 } qoc_precision;
typedef enum {
  QOC_TERM_ONE_BODY = 0,     /* coeff * sum_q w_q sigma_a^(q) over selected qubits */
  QOC_TERM_RING_PAIR = 1,    /* coeff * sum_{q=1..n} sigma_a^(q) sigma_b^(q+distance), indices mod n */
  QOC_TERM_ALL_PAIRS = 2,    /* coeff * sum_{q<q'} sigma_a^(q) sigma_b^(q') */
  QOC_TERM_PAULI_STRING = 3  /* coeff * prod_p sigma(x_p, z_p): (1,0)=X, (0,1)=Z, (1,1)=Y */
} qoc_term_kind;
typedef enum { QOC_SITES_ALL = 0, QOC_SITES_EVEN = 1, QOC_SITES_ODD = 2 } qoc_sites;

/* One Hermitian Pauli-sum term with a real coefficient (Sec. II A: H_x, H_y, H_z and the
 * ring coupling H_z,cpl; Eqs. (5)-(7)).  For ONE_BODY, w_q = (-1)^q when staggered,
 * else 1, and `sites` selects even, odd or all qubits q.  op_a/op_b are 'x','y','z'.
 * For PAULI_STRING, x_mask / z_mask are indexed by bit position p. */
typedef struct {
  int32_t kind;
  int32_t distance;
  int32_t sites;
  int32_t staggered;
  double coeff;
  char op_a;
  char op_b;
  char pad_[6];
  uint64_t x_mask;
  uint64_t z_mask;
} qoc_term;

typedef struct qoc_basis_s* qoc_basis;
typedef struct qoc_system_s* qoc_system;
typedef struct qoc_plan_s* qoc_plan;

/* Orbits and symmetry-adapted block table of the group (App. A, Eq. (A2); Table I).
 * n: 1..30 for DIHEDRAL/CYCLIC (basis states are enumerated on the device),
 * 1..4096 for SYMMETRIC (closed form, no enumeration).  stride must divide n
 * (ring groups); it is ignored for SYMMETRIC.  Orbit representatives are computed
 * on the device with integer arithmetic and the block sizes are cross-checked on
 * the host against the character formula; a mismatch returns QOC_ERR_NUMERIC.
 * Synchronises `stream` before returning. */
qoc_status qoc_build_basis(int n, int group, int stride, void* stream, qoc_basis* out);
void qoc_basis_free(qoc_basis basis);

/* Block table: writes up to `cap` entries of sizes m_theta and copies d_theta (host
 * arrays) and the number of blocks.  For SYMMETRIC, copies is 1 (one copy per J). */
qoc_status qoc_basis_blocks(qoc_basis basis, int* nblocks, int32_t* sizes, int32_t* copies, int cap);

/* Orbit representatives (host array, ascending): which = 0 for the orbits of the whole
 * group, 1 for the orbits of its rotation subgroup, 2 + b for the representatives that
 * index block b.  *count receives the total; at most `cap` are written. */
qoc_status qoc_basis_reps(qoc_basis basis, int which, uint64_t* reps, int64_t cap, int64_t* count);

/* Dense state (2^n interleaved complex128, device) -> block panels (device), and back
 * (App. A: the columns of the adjoint matrix are the basis states above).
 * Ring groups only; QOC_ERR_UNSUPPORTED for SYMMETRIC. */
qoc_status qoc_state_to_blocks(qoc_basis basis, const void* dense_dev, void* blocks_dev, void* stream);
qoc_status qoc_state_from_blocks(qoc_basis basis, const void* blocks_dev, void* dense_dev, void* stream);

/* Project H0 and the K control Hamiltonians into every block: H_theta = A_theta^dag H
 * A_theta (Sec. II A; Fig. 2's block structure).  h0 has n_h0 terms; hk holds the terms
 * of H_1..H_K back to back, n_hk[k] of them for H_k.  Every term is first checked for
 * exact invariance under the group generators on its integer bit masks; a term that
 * breaks the symmetry returns QOC_ERR_SYMMETRY before device work.  The system keeps
 * complex128 and complex64 copies of every block on the device.  K: 0..32.
 * Synchronises `stream` before returning. */
qoc_status qoc_project(qoc_basis basis, const qoc_term* h0, int n_h0, const qoc_term* hk,
                       const int* n_hk, int K, void* stream, qoc_system* out);
void qoc_system_free(qoc_system system);

/* Host-only exact check that the sum of `count` terms is invariant under the group
 * generators (rotation by `stride`, and the reflection for DIHEDRAL), compared on the
 * integer Pauli masks and exactly equal coefficients after merging equal strings
 * (Sec. II A: which sums carry S_n or D_n symmetry).  For SYMMETRIC, only uniform
 * one-body sums and all-pairs sums with equal letters are accepted.  Returns QOC_OK or
 * QOC_ERR_SYMMETRY (QOC_ERR_INVALID_ARG for malformed input).  n: 1..64 (ring groups). */
qoc_status qoc_check_symmetry(int n, int group, int stride, const qoc_term* terms, int count);

/* Copy block `block` of operator `op` (0 = H0, k = H_k) into a caller buffer as a dense
 * column-major m x m interleaved complex128 matrix (device). */
qoc_status qoc_system_block(qoc_system system, int block, int op, void* dst_dev, void* stream);

/* Execution plan for N slices of length dt at a precision (QOC_C128 or QOC_C64).
 * The plan fixes the Taylor degree menu, the Frechet-series length and the number of
 * propagator slices held at once (segment) so that the workspace stays within
 * max_workspace_bytes (0: 85 % of the free device memory, at most 240 GiB);
 * when the whole pulse does not fit, propagators are recomputed segment by segment in
 * the backward sweep.  u_bound > 0 bounds |u[j,k]| for every
 * call that uses this plan; the plan uses it, with the exact 1-norms of the blocks, to
 * bound dt*||H0 + sum u_k H_k||_1 by the triangle inequality.  A slice whose exact
 * 1-norm exceeds that bound (possible only when some |u| exceeds u_bound) makes the
 * hot-path call report QOC_ERR_NUMERIC.
 * Host-only apart from reading the free device memory and uploading small tables. */
qoc_status qoc_plan_create(qoc_system system, int precision, int N, double dt, double u_bound,
                           size_t max_workspace_bytes, qoc_plan* out);
/* One plan for P independent problems run together (the batched form of the same
 * computation: every block of every problem and every slice shares the launches).
 * Problem p uses systems[p] (systems may repeat, e.g. one Hamiltonian with many
 * candidate pulses), N[p] slices of length dt[p]; u_bound bounds every |u|.
 * The hot-path calls then take concatenated arrays, problem after problem:
 *   controls and gradients: [N[p]][K_p] float64 blocks back to back;
 *   psi0 / psi_f: each problem's panels (length D_p) back to back;
 *   objective output: [P][8] (layout of qoc_fidelity_grad's out_dev);
 *   propagators (qoc_propagate): per problem, per block, N[p] m x m matrices.
 * qoc_plan_info reports P, the number of (problem, block) jobs and the total lengths.
 * P: 1..65535.  Host-only. */
qoc_status qoc_plan_create_batched(const qoc_system* systems, int P, const int* N, const double* dt, int precision,
                                   double u_bound, size_t max_workspace_bytes, qoc_plan* out);
/* Execution plan over a subset of the system's blocks, in the order given (each index
 * once, 0 <= blocks[i] < number of blocks): only those blocks' propagators, states and
 * gradients are formed, and the caller's panels psi0 / psi_f hold only those blocks
 * (length sum of m * copies over the subset, in the given order; qoc_plan_info [13]).
 * The paper's runtime comparisons propagate the all-up and all-down states, which lie in
 * the first block (Sec. II B, Sec. III A: both states evolve inside the first subspace, so
 * the first block of each transformed operator is all the computation needs), so
 * blocks = {0} is that computation.  Other arguments and errors as qoc_plan_create;
 * QOC_ERR_INVALID_ARG for an empty, repeated or out-of-range block list.  Host-only. */
qoc_status qoc_plan_create_blocks(qoc_system system, const int* blocks, int nblocks, int precision, int N,
                                  double dt, double u_bound, size_t max_workspace_bytes, qoc_plan* out);
void qoc_plan_free(qoc_plan plan);
qoc_status qoc_plan_workspace_size(qoc_plan plan, size_t* bytes);
/* Plan facts: info[0] segment length, [1] number of segments, [2] Taylor degree step r,
 * [3] largest degree, [4] Frechet series terms, [5] Frechet sub-steps, [6] workspace
 * bytes per slice (propagator slot and Taylor scratch), [7] largest squaring count, [8] gradient chunk (slices), [9] GEMM
 * grid, [10] problems P, [11] (problem, block) jobs, [12] total controls (sum N_p K_p),
 * [13] total panel length (sum D_p), [14] total propagator entries, [15] GEMM tile
 * variant in use, [16] slices per Taylor-scratch chunk, [17] largest number of work-groups
 * sharing one block's sweep (1: one work-group per block), [18] problem groups, [19] powers
 * of the exponent formed by the generator instead of products (2: Y^2 and Y^3, for systems
 * with at most 4 controls; 0 otherwise), [20] planes per propagator slot (4: U and room for
 * the gate product tree; 2: U alone), [21] 1 when operator products are formed per call in
 * the workspace (qoc_set_products_policy).
 * Workspace: U of every slice of a segment (both sweeps read it: the backward one takes
 * U^dag lambda as dot products down U's columns), Taylor scratch (Y..Y^r and two ping-pong
 * buffers) of one chunk of slices, states, gradient slots; each slice's slot also holds
 * room for qoc_gate_propagate's product tree when every propagator still fits with it.  When the budget holds
 * everything, segment = chunk = N; when it holds every propagator and the scratch of at
 * least 8 slices, segment = N and the chunk is what the rest holds; otherwise the
 * propagators of earlier segments are recomputed during the backward sweep.
 * Batched plans: when the propagators of all problems do not fit the budget at once, the
 * problems are split into groups of consecutive problems whose propagators do fit, run one
 * after another in the same workspace (nothing is recomputed for them); a problem too large
 * on its own forms a group that segments.  [0], [1], [8] and [16] then describe the group
 * with the most segments; qoc_plan_groups lists every group. */
qoc_status qoc_plan_info(qoc_plan plan, int64_t* info, int cap);
/* Problem groups of a plan (see qoc_plan_info): *count groups (1 for a plan without
 * groups); for each of the first `cap`, its first problem, segment length and number of
 * segments (host arrays; any may be NULL).  Host-only. */
qoc_status qoc_plan_groups(qoc_plan plan, int* count, int32_t* prob_begin, int32_t* seg_len, int32_t* nseg, int cap);

/* GEMM tile variants.  The propagator and panel GEMMs are compiled for 3 work-group tile
 * shapes per precision (qoc_variant_name: e.g. "fp32 128x64"); every shape accumulates
 * each output element in the same order, so results do not depend on the choice.  A new
 * plan uses variant 0.  qoc_plan_set_variant selects one (host call; synchronises the
 * device).  qoc_plan_autotune times every variant on the plan's own work (the first
 * segment's propagators for controls u_dev, plus one gradient panel GEMM) with HIP
 * events on `stream`, keeps the fastest and returns its index in *chosen and, when
 * times_ms is not null, each variant's time (ms, 3 entries).  It synchronises and uses
 * the caller's workspace as scratch; the plan's results are unchanged. */
qoc_status qoc_plan_set_variant(qoc_plan plan, int variant);
const char* qoc_variant_name(int precision, int variant);
qoc_status qoc_plan_autotune(qoc_plan plan, const double* u_dev, void* workspace, size_t workspace_bytes,
                             void* stream, int* chosen, double* times_ms);

/* Slice propagators U_j (Eq. (3)) for every block and slice: scaled Taylor polynomial
 * (Paterson-Stockmeyer) with repeated squaring, matrix products on the MFMA units.
 * U_out_dev receives, block after block, N column-major m x m interleaved complex128
 * matrices (slice-major within a block).  Requires a plan whose segment covers N. */
qoc_status qoc_propagate(qoc_plan plan, const double* u_dev, void* U_out_dev, void* workspace,
                         size_t workspace_bytes, void* stream);

/* Objective and exact gradient (Eqs. (3)-(4); App. B, Eq. (B2) taken to all orders).
 * psi0_dev, psif_dev: block panels (interleaved complex128, length D).
 * out_dev (float64, 8 entries): [0] F = |o|^2 / (||psi_N||^2 ||psi_f||^2),
 * [1] |o|^2, [2] Re o, [3] Im o with o = <psi_f|psi_N>, [4] ||psi_N||^2,
 * [5] ||psi_f||^2, [6] largest squaring count used (by all problems of the call, or of the
 * problem's group when a batched plan has problem groups), [7] status flags (0 = clean;
 * bit 0: a slice exceeded the plan's norm bound; bit 1: non-finite value; bit 2: a
 * co-operative sweep's hand-off between work-groups stalled and the sweep gave up, so
 * the outputs are invalid).
 * grad_dev (float64 [N][K]) receives dF/du[j,k] = 2 Re(conj(o) do/du[j,k]) /
 * (||psi_N||^2 ||psi_f||^2).  For a batched plan every array concatenates the
 * problems in plan order (u and grad: N_p x K_p each; panels: D_p each) and out_dev
 * holds 8 entries per problem.  Fully asynchronous (no host synchronisation), so the
 * call can be captured into a HIP graph. */
qoc_status qoc_fidelity_grad(qoc_plan plan, const double* u_dev, const void* psi0_dev,
                             const void* psif_dev, double* out_dev, double* grad_dev,
                             void* workspace, size_t workspace_bytes, void* stream);

/* Objective only (Eqs. (3)-(4)): the propagators and the forward sweep, segment by
 * segment, then o = <psi_f|psi_N> and F, with no backward sweep and no gradient.  Each
 * propagator is used once, so a plan with several segments recomputes nothing here.
 * Arguments, out_dev layout (8 float64 per problem, status bits 0-2 as for
 * qoc_fidelity_grad), batching and asynchrony as qoc_fidelity_grad. */
qoc_status qoc_fidelity(qoc_plan plan, const double* u_dev, const void* psi0_dev, const void* psif_dev,
                        double* out_dev, void* workspace, size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, hosts that forbid hipMalloc): qoc_fidelity_grad with its workspace taken
 * from a static device array of QOC_STATIC_SCRATCH_BYTES (64 MiB) that the library's code
 * object holds on every GPU it runs on until the process ends.  The call allocates nothing
 * (no hipMalloc / hipFree or allocating library routine); the caller still passes the
 * inputs and outputs, laid out as for qoc_fidelity_grad, with the same results.  The plan's
 * workspace must fit (create it with max_workspace_bytes <= QOC_STATIC_SCRATCH_BYTES; a
 * smaller budget only means more segments), else QOC_ERR_OUT_OF_MEMORY before any device
 * work.  Every call on one GPU shares that GPU's array and leaves its contents behind;
 * what a call needs zeroed it clears itself.  Calls that overlap on one GPU (two streams,
 * two threads, or this call beside a qoc_fidelity_grad_noalloc of another plan) race on
 * the array: serialise them.  Asynchronous on `stream`, like qoc_fidelity_grad. */
#define QOC_STATIC_SCRATCH_BYTES (64ull << 20)
qoc_status qoc_fidelity_grad_noalloc(qoc_plan plan, const double* u_dev, const void* psi0_dev, const void* psif_dev,
                                     double* out_dev, double* grad_dev, void* stream);

/* One state of the sweeps of the last qoc_fidelity_grad (or, for which = 0, qoc_fidelity)
 * call that used `workspace` with this plan (Eq. (3): psi_{j+1} = U_j psi_j; App. B:
 * lambda_j = U_j^dag lambda_{j+1}, lambda_N = psi_f): which = 0 the forward state psi_j,
 * 0 <= j <= N; which = 1 the costate lambda_j, 1 <= j <= N.  Then o = <lambda_j|psi_j>
 * for every j, and changing u[j-1, k] alone changes o to <lambda_j| U_{j-1}(u') |psi_{j-1}>.
 * out_dev receives problem `problem`'s block panels (interleaved complex128, length D_p,
 * the layout of psi0_dev), in the working precision of the plan converted to FP64.
 * QOC_ERR_INVALID_ARG for an index out of range.  Asynchronous on `stream`. */
qoc_status qoc_plan_read_state(qoc_plan plan, int problem, int which, int j, const void* workspace,
                               size_t workspace_bytes, void* out_dev, void* stream);

/* Co-operative sweep switches, for tests of its fallback and failure handling (0 in
 * normal use).  QOC_SWEEP_SOLO: every block whose rows span several work-groups is swept
 * by one work-group alone (the path the sweep takes by itself when its groups are not all
 * resident); results are unchanged.  QOC_SWEEP_TEST_STALL_FWD / _BWD: the forward or
 * backward sweep's hand-offs wait for tags that are never written, so each bounded wait
 * times out (tens of milliseconds per group) and the call reports status bit 2 (outputs
 * invalid), as after a real stall.  They act only on plans whose sweeps run co-operatively.
 * Host call. */
enum { QOC_SWEEP_SOLO = 1, QOC_SWEEP_TEST_STALL_FWD = 2, QOC_SWEEP_TEST_STALL_BWD = 4 };
qoc_status qoc_plan_set_sweep_mode(qoc_plan plan, int mode);

/* Generator switch, for tests (0 in normal use).  The slice generator (Eq. (3)'s exponent
 * and, with operator products, its powers and first Taylor combinations) runs one
 * work-group per (block, group of 8 slices), split over column ranges when there are fewer
 * than 16 such pairs per compute unit.  ranges = 0 keeps that rule; ranges >= 1 runs every
 * call over exactly min(ranges, max(1, widest padded block / 16)) ranges (1: unsplit).
 * Each element is formed by the same arithmetic either way, so results are unchanged bit
 * for bit.  QOC_ERR_INVALID_ARG for a null plan or ranges < 0.  Host call. */
qoc_status qoc_plan_set_generator_split(qoc_plan plan, int ranges);

/* Gate propagation: the unitary a pulse implements, K = U_{N-1} ... U_1 U_0 (Eq. (3)'s
 * slice propagators in time order), for every block of a one-problem plan; Sec. III B
 * compares two such products by the gate fidelity below.  The propagators are formed as
 * in qoc_propagate and multiplied as a balanced tree of batched complex GEMMs on the MFMA
 * units (log2 N levels, N - 1 products per block).  K_out_dev receives, block after
 * block, column-major m x m interleaved complex128 matrices (length sum of m^2).
 * Requires every propagator of the pulse to fit the plan's workspace twice over (one
 * segment with room for the tree: qoc_plan_info [1] == 1 and [20] == 4), else
 * QOC_ERR_UNSUPPORTED; QOC_ERR_UNSUPPORTED for a batched
 * plan.  Like qoc_propagate it reports no status word: qoc_plan_slice_stats or
 * qoc_fidelity_grad flag controls beyond the plan's norm bound.  Asynchronous on
 * `stream`; uses the workspace as qoc_fidelity_grad does. */
qoc_status qoc_gate_propagate(qoc_plan plan, const double* u_dev, void* K_out_dev, void* workspace,
                              size_t workspace_bytes, void* stream);
/* Gate fidelity of two block-diagonal unitaries in the layout qoc_gate_propagate writes:
 * t = sum_blocks d Tr(Ka^dag Kb) with d the block's copies (2 for E_m, 1 otherwise),
 * na = sum_blocks d ||Ka||_F^2, nb likewise, D = sum_blocks d m, and F = |t|^2 / (na nb).
 * For unitaries na = nb = D, so F is Sec. III B's |Tr(K_a^dag K_b) / 2^n|^2 when the plan
 * covers every block of a ring group (D = 2^n); over a subset of blocks it is the same
 * quantity restricted to their subspace; for S_n blocks each J carries weight 1.  The
 * norms keep the drift of reduced-precision products (K slightly off unitary) out of F.
 * out_dev (float64, 6 entries): [0] F, [1] Re t, [2] Im t, [3] D, [4] na, [5] nb.  FP64,
 * fixed-order sums; the first 2 KB per block of the workspace hold partial sums.
 * Asynchronous. */
qoc_status qoc_gate_fidelity(qoc_plan plan, const void* Ka_dev, const void* Kb_dev, double* out_dev,
                             void* workspace, size_t workspace_bytes, void* stream);

/* Trotterised propagator for per-qubit controls (Sec. III B, Eqs. (8)-(11)) on the Ising
 * ring H_j = sum_i [(B_z/2) sz_i + (Bx_i[j] sx_i + By_i[j] sy_i)/2]
 *          + (c_cpl/4) sum_i sz_i sz_{i+1}  (qubit n+1 = qubit 1):
 *   U_j^LTS = prod_{i=1..n} [exp(-i dt (H_0^(i) + H_c'^(i)[j])) exp(-i (dt/n) H_cpl)],
 * the product written i = 1 leftmost, so qubit n's bracket acts first and, inside a
 * bracket, the coupling factor first.  qoc_lts_apply computes
 * psi_out = U_{N-1}^LTS ... U_0^LTS psi_in for ncols state columns.
 * n: 1..13 (each column is held in LDS; QOC_ERR_UNSUPPORTED beyond).  u_dev: float64
 * [N][2n] device controls, u[j][2(i-1)] = Bx_i, u[j][2(i-1)+1] = By_i.  psi_in_dev:
 * column-major 2^n x ncols interleaved complex128 in the computational basis (qubit q at
 * bit n - q, bit 0 = spin up), or NULL for the identity columns 0 .. ncols - 1 (ncols <=
 * 2^n), which yields those columns of K^LTS = U_{N-1}^LTS ... U_0^LTS.  psi_out_dev: the
 * same layout (2^n x ncols).  workspace: caller-owned device memory of at least
 * qoc_lts_workspace_size(n, N) bytes (the 2 x 2 factors of every slice and qubit).  FP64;
 * one work-group per column; asynchronous on `stream`. */
qoc_status qoc_lts_workspace_size(int n, int N, size_t* bytes);
qoc_status qoc_lts_apply(int n, double Bz, double c_cpl, const double* u_dev, int N, double dt,
                         const void* psi_in_dev, int ncols, void* psi_out_dev, void* workspace,
                         size_t workspace_bytes, void* stream);
/* State transfer through the same Trotterised propagator and its exact gradient, for P
 * independent problems (App. B: the transformed propagator serves gradient-based methods;
 * here each qubit factor is differentiated exactly, not to first order).  Problem p has
 * controls u_dev[p] (float64 [N][2n], problems back to back), psi0_dev[p] and psif_dev[p]
 * (2^n interleaved complex128 each, back to back).  out_dev (float64 [P][8]): F =
 * |o|^2 / (||psi_N||^2 ||psi_f||^2), |o|^2, Re o, Im o, ||psi_N||^2, ||psi_f||^2, 0, status
 * (bit 1: non-finite), o = <psi_f|psi_N>.  grad_dev (float64 [P][N][2n]): dF/du =
 * 2 Re(conj(o) <lambda| dg/du |psi>) / norms, psi the state just before the factor g of
 * that control and lambda the costate just after it.  n: 1..12 (state and costate in LDS;
 * QOC_ERR_UNSUPPORTED beyond).  workspace: qoc_lts_grad_workspace_size(n, N, P) bytes (the
 * factors and their derivatives).  FP64; one work-group per problem; the backward pass
 * recovers the states by undoing each factor, so nothing is stored per slice.
 * Asynchronous on `stream`. */
qoc_status qoc_lts_grad_workspace_size(int n, int N, int P, size_t* bytes);
qoc_status qoc_lts_fidelity_grad(int n, double Bz, double c_cpl, const double* u_dev, int N, double dt,
                                 int P, const void* psi0_dev, const void* psif_dev, double* out_dev,
                                 double* grad_dev, void* workspace, size_t workspace_bytes, void* stream);

/* Where plans created from now on take the operator products of systems with at most 4
 * controls (process-wide, host call).  0 (default): a plan forms the products its systems
 * lack and keeps them with the systems when they fit an eighth of the free device memory;
 * otherwise (a large batch of distinct Hamiltonians) the products of the systems without
 * them are formed at the start of every hot-path call into the plan's workspace (counted in
 * qoc_plan_workspace_size), in the plan's precision, group by group for plans with problem
 * groups.  1: always the workspace form for systems that keep no products (for tests of
 * that form).  QOC_ERR_INVALID_ARG for another value. */
qoc_status qoc_set_products_policy(int policy);

/* Progress lines for long batched calls (process-wide switch, off by default).  When
 * enabled, every call on a plan with problem groups (qoc_plan_groups) queues after each
 * group a host function on the call's stream that prints, once the group's work has
 * finished, "[qoc] problem group g/G done (problems a..b)" to stderr.  For callers that
 * watch a long call's liveness; it adds one host callback per group and is not meant for
 * graph capture.  Always QOC_OK. */
qoc_status qoc_set_progress(int enable);

/* Benchmark instrumentation (process-wide, not thread-safe while enabled).
 * qoc_profile_begin pre-creates HIP events for up to max_launches kernel launches and
 * enables recording: every kernel the hot-path calls enqueue is bracketed by events on
 * the launch stream.  qoc_profile_end synchronises on them, disables recording and
 * writes, per kernel kind, the summed duration in milliseconds and the launch count:
 * [0] generator + norm, [1] propagator GEMM (powers, Horner or degree-12 steps,
 * squarings), [2] gate product tree (qoc_gate_propagate),
 * [3] forward sweep, [4] backward sweep, [5] objective, [6] gradient GEMM, [7] gradient
 * vector kernels, [8] gradient reduction, [9] other.  qoc_profile_end returns
 * QOC_ERR_INVALID_ARG (after writing the partial totals) when more launches were made than
 * max_launches covers. */
qoc_status qoc_profile_begin(int max_launches);
/* Measured matrix-core rate of the current device for the MFMA instruction the tiles use
 * (v_mfma_f32_16x16x4f32 for QOC_C64, v_mfma_f64_16x16x4f64 for QOC_C128): every wave of a
 * full grid issues independent MFMAs on register operands, with no memory traffic; *tflops
 * receives 2 * 16 * 16 * 4 flops per instruction over the time of one launch (HIP events on
 * `stream`, after a warm-up).  The reference for the propagator GEMM's fraction of the
 * achievable rate.  Synchronises `stream`. */
qoc_status qoc_measure_mfma_peak(int precision, double* tflops, void* stream);
qoc_status qoc_profile_end(double* ms, int64_t* launches, int cap);

/* Per job and slice (host arrays [jobs][max N], jobs = (problem, block) pairs in order):
 * the evaluation the plan's propagators pick for these controls (the algorithmic work of
 * Eq. (3)'s exponentials): q >= 1 for Paterson-Stockmeyer Taylor of degree q * r
 * ((r - 1) + (q - 1) matrix products), q = 0 for the four-product degree-12 Taylor
 * evaluation (Bader, Blanes & Casas 2019); squaring count s; FP64 norm
 * dt*||H0 + sum_k u[j,k] H_k||_1.  Entries beyond a problem's N: q = -1, s = 0, norm 0.
 * Synchronises `stream`. */
qoc_status qoc_plan_slice_stats(qoc_plan plan, const double* u_dev, int32_t* q, int32_t* s, double* norms,
                                void* stream);

/* GRAPE pulse optimisation: GRAPE raises the objective by gradient steps on every slice
 * sample (Sec. I), with the gradient of App. B (here the exact one of qoc_fidelity_grad).
 * The paper's update rule is in its Supplementary Material; this entry point uses
 * limited-memory BFGS ascent on F(u) (Nocedal, Math. Comp. 1980) with a backtracking
 * Armijo line search:
 *   direction d = H g by the two-loop recursion over the last `memory` kept pairs
 *   s = u_new - u_old, y = g_old - g_new (g = dF/du), H0 = (s.y / y.y) I from the newest
 *   pair; with no pair d = (step0 / max|g|) g; a pair is kept when
 *   s.y > 1e-10 sqrt(s.s y.y); the memory is cleared when g.d <= 0; trials u + alpha d
 *   with alpha = 1, 1/2, ... (up to max_backtrack halvings) are accepted when the
 *   evaluation's status word is 0 and F(u + alpha d) >= F(u) + c1 alpha g.d.
 * Stops when F >= f_target (reason QOC_OPT_TARGET), max|g| <= gtol (QOC_OPT_GTOL), after
 * max_iter accepted steps (QOC_OPT_MAX_ITER) or when a line search accepts no trial
 * (QOC_OPT_LINE_SEARCH_FAILED).  memory: 1..64; c1 in (0, 1); step0 > 0;
 * max_backtrack: 0..60; max_iter >= 0.
 * plan: a one-problem plan (QOC_ERR_UNSUPPORTED otherwise).  u_dev: float64 [N][K] device
 * controls, the start on entry and the last accepted point on return.  psi0_dev /
 * psif_dev: as for qoc_fidelity_grad.  workspace: caller-owned device memory of at least
 * qoc_optimize_workspace_size(plan, memory, &bytes) bytes; its first
 * qoc_plan_workspace_size bytes serve the evaluations, the rest holds the pairs and
 * vectors (about (2 memory + 6) N K doubles).  hist_host (host, hist_cap entries): F at
 * the start and after every accepted step, as many as fit.  result: accepted steps,
 * objective evaluations, stop reason and the final F.  The direction, trial point and pair
 * updates run as FP64 kernels with fixed-order reductions; the line search decides on the
 * host, so the call synchronises `stream` after every evaluation and cannot be captured.
 * A trial outside the plan's norm bound (status bit 0) or with a non-finite value counts as
 * rejected.  QOC_ERR_NUMERIC if the start is not a clean evaluation or a co-operative sweep
 * stalls. */
typedef struct qoc_lbfgs_options {
  int max_iter;
  int memory;
  double step0;
  double c1;
  int max_backtrack;
  double f_target;
  double gtol;
} qoc_lbfgs_options;
typedef struct qoc_lbfgs_result {
  int iterations;
  int evaluations;
  int reason;
  double F;
} qoc_lbfgs_result;
enum { QOC_OPT_TARGET = 0, QOC_OPT_GTOL = 1, QOC_OPT_MAX_ITER = 2, QOC_OPT_LINE_SEARCH_FAILED = 3 };
qoc_status qoc_optimize_workspace_size(qoc_plan plan, int memory, size_t* bytes);
/* The same L-BFGS iterations on the Trotterised per-qubit-control objective of
 * qoc_lts_fidelity_grad (one problem: n, B_z, c_cpl, N, dt, u_dev [N][2n], psi0_dev /
 * psif_dev of 2^n amplitudes as there).  There is no plan norm bound: a trial is
 * rejected only when its evaluation is not finite.  workspace: at least
 * qoc_optimize_lts_workspace_size(n, N, memory) bytes.  Options, history, result, errors
 * and synchronisation as qoc_optimize_lbfgs. */
qoc_status qoc_optimize_lts_workspace_size(int n, int N, int memory, size_t* bytes);
qoc_status qoc_optimize_lbfgs_lts(int n, double Bz, double c_cpl, int N, double dt,
                                  const qoc_lbfgs_options* options, double* u_dev, const void* psi0_dev,
                                  const void* psif_dev, void* workspace, size_t workspace_bytes, void* stream,
                                  double* hist_host, int hist_cap, qoc_lbfgs_result* result);
qoc_status qoc_optimize_lbfgs(qoc_plan plan, const qoc_lbfgs_options* options, double* u_dev,
                              const void* psi0_dev, const void* psif_dev, void* workspace,
                              size_t workspace_bytes, void* stream, double* hist_host, int hist_cap,
                              qoc_lbfgs_result* result);

/* Status text and the calling thread's last error detail. */
const char* qoc_status_string(qoc_status status);
const char* qoc_last_error(void);
/* Library version (major*10000 + minor*100 + patch). */
int qoc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QOC_H */
