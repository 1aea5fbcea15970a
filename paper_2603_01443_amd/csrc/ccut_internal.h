// Internal definitions shared by the host planner and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "ccut.h"

namespace ccut {

// MFMA merge GEMM variants (0..3 tiled, 4 R-stationary, 5 LDS-staged; see merge_mfma.h)
constexpr int MERGE_VARIANTS = 7;

// ----------------------------------------------------------------- errors
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
int hip_fail(hipError_t e, const char* what);

#define CCUT_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return ::ccut::hip_fail(e_, #call); \
  } while (0)

using cd = std::complex<double>;

// ------------------------------------------------------- register-level ops
// A gate program on an m-qubit register after single-qubit fusion.
enum HOpKind : int32_t { HOP_1Q = 0, HOP_CZ = 1, HOP_CX = 2 };

struct HOp {
  int32_t kind;
  int32_t q0, q1;  // 1Q: q0 only.  CX: q0 = control, q1 = target
  bool diag;       // 1Q matrix is diagonal
  int32_t slot;    // -1, or the variant bit choosing m[1] over m[0]
  cd m[2][4];      // row-major 2x2 (m00, m01, m10, m11) for slot bit 0 / 1
};

struct Program {
  int32_t nq = 0;
  std::vector<HOp> ops;
};

// ------------------------------------------------------- gate kinds
bool is_two_qubit_kind(int kind);
// SWAP, iSWAP, RXX, RYY, RZZ: each is phase * exp(-i/2 (tx XX + ty YY + tz ZZ))
bool is_pauli_rotation_kind(int kind);
void pauli_rotation_form(const ccut_gate_t& g, double t[3], cd* phase);
// exp(-i/2 (t0 XX + t1 YY + t2 ZZ)) = sum_P c[P] P (x) P with P = I, X, Y, Z (the
// three rotations commute; expanding cos(t/2) - i sin(t/2) PP and using
// XX YY = -ZZ and its cyclic forms gives the four coefficients)
void pauli_rotation_coeffs(const double t[3], cd c[4]);
// Validates gate k of a circuit on q qubits (kind and qubit indices).
int check_gate(const ccut_gate_t& g, int q, int64_t k);

// Append a single-qubit matrix, fusing it into the previous single-qubit op on
// that qubit when every op in between on the qubit commutes with it.
struct ProgramBuilder {
  Program prog;
  std::vector<int32_t> last1q;   // index of the last 1Q op per qubit, -1 if none
  std::vector<uint8_t> any_since, nondiag_since;
  explicit ProgramBuilder(int nq);
  void one_qubit(int t, const cd m0[4], const cd m1[4], int slot);
  void cz(int a, int b);
  void cx(int c, int t);
  // Any gate of the circuit whose qubits all lie in this register (qubit indices
  // minus `off`); the Pauli-rotation kinds go through exact CX decompositions.
  void gate(const ccut_gate_t& g, int off);
};

// --------------------------------------------------------- device op format
enum KOpType : int32_t {
  KOP_DENSE = 0,   // 2x2 on local bit a
  KOP_DIAG = 1,    // diag(m0, m3) on local bit a
  KOP_CZL = 2,     // sign flip where sum_t popcount(i & (i >> shift_t) & mask_t) is odd;
                   // in register stages the header repeats terms 0 and 1 in (a, b) and
                   // (pad[0], pad[1]), so that the 32-byte header read brings them
  KOP_SCALAR = 3,  // multiply the block by m0 (bit a of the block base is 0) or m3 (it is 1)
  KOP_CXL = 4,     // CX with local control a, local target b
  KOP_GROUP = 5,   // register stages only: one 2x2 gate per register position (gates on
                   // distinct qubits commute); the KOP_DENSE records of positions
                   // 0..REG_BITS-1 follow (identity where the group has no gate), and
                   // the header repeats their variant slots in b, slot, cond, nterms so
                   // that one 32-byte read gives every matrix address.  pad[0]: first
                   // MFMA operand table of the group, pad[1]: number of members with a
                   // slot (the group has 2^pad[1] tables, one per choice of those slots)
  KOP_FUSED = 6,   // register stages only: the a records that follow (groups, and
                   // diagonal, CZ and CX ops confined to the register bits) form one
                   // 16x16 matrix on the register positions.  The MFMA path applies that
                   // matrix from its operand tables and skips the records; the float32
                   // path skips this header and runs the records one by one.  b, slot,
                   // cond, nterms: the distinct variant slots of the records (the
                   // first k valid, the rest -1), so that table choice bit j is slot j;
                   // pad[0]: first operand table, pad[1]: number of slots; m[0..3] (as
                   // int32): the local bit of each register position
};

constexpr int KOP_MAX_TERMS = 8;
constexpr int FUSED_MAX_RECORDS = 48;  // records of one KOP_FUSED run (staged in LDS to build its table)

struct KOp {
  int32_t type;
  int32_t a, b;
  int32_t slot;   // -1 or variant bit selecting m[8..15] over m[0..7]
  int32_t cond;   // -1, or register qubit whose bit in the block base must be 1
  int32_t nterms; // KOP_CZL term count
  int32_t pad[2];
  float m[16];    // (re, im) of m00, m01, m10, m11 per slot; KOP_CZL: uint32 (shift, mask) pairs
};
static_assert(sizeof(KOp) == 96, "KOp layout");

constexpr int PASS_MAX_B = 14;   // 2^14 complex64 = 128 KiB of LDS per block
constexpr size_t SIM_LDS_MAX = 160 * 1024;  // LDS of one compute unit (gfx950)
constexpr int REG_BITS = 4;      // amplitudes held per thread in a register stage: 2^4
constexpr int STAGE_MIN_B = 9;   // blocks of at least 2^9 amplitudes run in register stages

// A register stage inside an LDS block: every thread holds the 2^REG_BITS
// amplitudes spanned by local bits reg[] (ascending); thread slot t takes the
// other local bits in order, i.e. t with a zero inserted at each reg[] bit.
// Amplitude e of a thread sits at local index base | roff[e] and LDS slot
// pad(base) + proff[e] (the padding is additive over disjoint bits).  Ops of a
// stage: KOP_DENSE.a and KOP_CXL.b name register positions (0..REG_BITS-1);
// every other bit field is a local bit.  The kernel reads the first 32 bytes
// and forms roff / proff from reg[] itself.
struct StageDesc {
  int32_t op_begin;
  int32_t op_count;
  int32_t reg[REG_BITS];
  int32_t pad[2];
  int32_t roff[1 << REG_BITS];
  int32_t proff[1 << REG_BITS];
};
static_assert(sizeof(StageDesc) == 160, "StageDesc layout");

// MFMA form of a KOP_GROUP or KOP_FUSED run (split-float16 register-stage path).
// Its records form a 16x16 complex matrix G (for a group, the Kronecker product of
// its gates; position p = bit p of the row and column index) acting on a thread's
// 16 amplitudes.  As a real
// 32x32 matrix on (Re x[0..15], Im x[0..15]) it is the A operand of two
// v_mfma_f32_32x32x16_f16 steps (k = 0..15: real parts, 16..31: imaginary).
// Its output rows interleave the parts: row 2 e = Re y_e, row 2 e + 1 = Im y_e.
// A table holds, per lane l (row m = l % 32, k half h = l / 32), four uint4:
// hi and lo float16 parts of A[m][16 s + 8 h + e], e = 0..7, for s = 0, 1.
struct GroupRef {
  int32_t op;   // GROUP or FUSED header in the op table
  int32_t sel;  // bit j: choice of the j-th variant slot named in the header
};
constexpr int GROUP_TABLE_UINT4 = 64 * 4;  // uint4 per table (4 KiB)
constexpr float SIM_MFMA_SCALE = 16384.0f;  // 2^14: state scale inside a pass on the MFMA path

// One LDS-blocked pass over a state: blocks of 2^b amplitudes spanning the
// register qubits group[0..b); the other qubits are fixed per block.
struct PassDesc {
  int32_t b;         // local bits
  int32_t nq;        // register qubits
  int32_t op_begin;  // into the op table
  int32_t op_count;
  int32_t init;      // 1: the state is |0...0> before this pass (nothing is read)
  int32_t n_blocks;  // 2^(nq - b)
  int32_t stage_begin;  // into the stage table; stage_count == 0: ops run one by one
  int32_t stage_count;
  int32_t group[24]; // local bit j -> register qubit
  int32_t fixed[24]; // j-th non-group qubit (ascending), takes bit j of the block id
  int32_t from_src;  // 1: read the job's source state (SimJob::src_off) instead of its own
  int32_t pad;
};

struct Pass {
  std::vector<int32_t> group;  // size b, low qubits first
  std::vector<KOp> kops;       // block-level ops (local bits)
  bool init = false;
  bool from_src = false;
};

// Splits a pass's block-level ops into register stages (stage-level op encoding).
// fuse: fold what acts on a stage's register bits alone into KOP_FUSED runs.  Their
// operand tables are composed on the device at each call, which pays where a
// program's tables serve much work (the uncut passes) rather than per-call plans.
void stage_kops(const std::vector<KOp>& kops, int b, std::vector<StageDesc>& stages, std::vector<KOp>& out,
                bool fuse);

// Schedule a program into LDS-blocked passes of at most 2^bmax amplitudes.
// Low qubits [0, low_bits) sit in every block (coalesced runs).  The first pass
// starts from |0...0> (from_zero) or from a source state the job names.  A pass
// whose register-stage records would not fit in LDS beside its block (fuse: as
// stage_kops builds them) is split into consecutive passes over the same qubits.
int schedule_passes(const Program& prog, int bmax, int low_bits, std::vector<Pass>& out, bool from_zero = true,
                    bool fuse = false);

// A launch entry: one state (or a batch position) processed by one pass.
struct SimJob {
  uint64_t state_off;  // complex64 elements from the launch base pointer
  uint64_t src_off;    // state read by a from_src pass (prefix sharing: the parent state)
  int32_t pass_id;     // into the PassDesc table
  int32_t variant;
  int32_t wg_begin;    // first workgroup of this job in the launch
  int32_t pad;
};

// ------------------------------------------------------------- merge stage
// out[beta][y * NX + x] = sum_k w_k A(beta, k)[x] B(beta, k)[y]
struct MergeStage {
  int32_t K;             // terms
  int32_t batch;         // independent outputs
  int32_t qx, qy;        // log2 NX, log2 NY
  int32_t a_src, b_src;  // buffer ids: 0 = arena states, 1 = temp ping, 2 = temp pong, 3 = psi
  int32_t out_dst;
  int32_t weight_off;    // into the weight table (K entries)
  uint64_t a_off, b_off, out_off;          // complex64 elements from the buffer base
  uint64_t a_kstride, a_bstride, b_kstride, b_bstride, out_bstride;  // complex64 elements
};

// --------------------------------------------------------- device launches
// Device copies of a plan's tables, packed into one allocation.
struct DeviceTables {
  int device = -1;
  void* blob = nullptr;
  KOp* ops = nullptr;
  PassDesc* passes = nullptr;
  StageDesc* stages = nullptr;
  SimJob* jobs = nullptr;
  float* weights = nullptr;    // complex64 merge weights
  GroupRef* grefs = nullptr;   // MFMA operand tables to build (one per group and slot choice)
};

// ---------------------------------------------------------------- timing
enum ProfKernel : int { PROF_SIM = 0, PROF_MERGE_F32, PROF_SPLIT, PROF_TABLES, PROF_MERGE_GEMM, PROF_REDUCE,
                        PROF_MLP, PROF_EXPECT, PROF_N };
int prof_begin(int kernel, hipStream_t s);   // -1 when timing is off
void prof_end(int token, hipStream_t s);

struct ProfScope {
  int tok;
  hipStream_t s;
  ProfScope(int kernel, hipStream_t st) : tok(prof_begin(kernel, st)), s(st) {}
  ~ProfScope() { prof_end(tok, s); }
};

// Runs workgroups [wg_offset, wg_offset + total_wg) of a job list; grid_cap > 0
// makes the launch persistent (each workgroup loops over several blocks).
// gtab != nullptr selects the split-float16 MFMA path for register-stage groups
// (operand tables built by launch_group_tables); nullptr keeps float32 VALU.
// rec_cap: the most op records plus register stages of any pass the launch runs
// (the kernel copies a pass's op headers and stage heads to LDS, 32 bytes each).
int launch_sim(const SimJob* d_jobs, int n_jobs, int total_wg, int wg_offset, const PassDesc* d_passes,
               const StageDesc* d_stages, const KOp* d_ops, const uint4* gtab, float* base, int bmax,
               int rec_cap, int threads, int grid_cap, hipStream_t s);
// LDS bytes of a simulation workgroup with that capacity.
size_t sim_shmem_bytes(int bmax, int rec_cap);

// Copies `bytes` (a multiple of 16, 16-byte aligned) from pinned host memory to dst.
int launch_table_copy(void* dst, const void* host_src, uint64_t bytes, hipStream_t s);

// Builds the n MFMA operand tables listed by refs into gtab (n * GROUP_TABLE_UINT4 uint4).
int launch_group_tables(const KOp* d_ops, const GroupRef* d_refs, int n, uint4* gtab, hipStream_t s);

int launch_merge_f32(const MergeStage& st, const float* A, const float* B, float* out,
                     const float* d_weights, hipStream_t s);

// Pauli-string matrices of one segment's variant states (expectation values)
struct GramShape {
  int tm;      // tile side: 16, 32 or 64 entries
  int splits;  // amplitude-range splits, each writing a partial V x V matrix
};
GramShape gram_shape(int V, uint64_t N);
// out (V x V complex128) = sum over the splits of part[s], part: splits * V * V complex128
int launch_gram(const float2* states, int V, uint64_t N, uint32_t flip, uint32_t zy, GramShape g, double2* part,
                double2* out, hipStream_t s);

// Partial blocks of the float64 reductions (5 doubles each); every state size uses at most this many.
constexpr int RED_BLOCKS = 1024;
int launch_reduce(const float* psi, const float* ref, uint64_t n, double* d_partials, int n_blocks,
                  double* d_out, hipStream_t s);
// Device address of the fixed reduction scratch array on the current device (looked
// up once per device) and its capacity in doubles.
int reduce_scratch(double** out, uint64_t* n_doubles);

}  // namespace ccut
