/*
 * ccut.h - C ABI of the MI355X (gfx950) circuit-cutting library.
 *
 * The library reproduces the classical state-vector pipeline of
 * "Applicability and Limitations of Quantum Circuit Cutting in Classical
 * State-Vector Simulation" (arXiv 2603.01443):
 *
 *   T_cut = T_pre + T_sub + T_merge               (Sec. III.A, Eq. runtime_decomp)
 *   cut_plan            - preprocessing           (Appendix B, Algorithm 1)
 *   simulate_subcircuits- subcircuit simulation   (Appendix B, Algorithm 2)
 *   merge_full_state    - full-state merging      (Appendix B, Algorithm 3)
 *   simulate_uncut      - the uncut baseline T_orig = O(2^q D) (Sec. III.A)
 *
 * Every cross-segment CZ is cut with the rank-2 decomposition of Eq. (CZ),
 *   CZ = (S (x) S + i S^dag (x) S^dag) / (1 + i),   S = diag(1, i),
 * and every cross-segment CX through CX = (I (x) H) CZ (I (x) H) (Sec. II.A.2),
 * so the target side of a cut CX receives H S H or H S^dag H.  The other
 * two-qubit kinds (SWAP, iSWAP, RXX, RYY, RZZ) are cut through their
 * operator-Schmidt decomposition, Eq. (schmidt), with k = 2 or 4 terms.
 *
 * Conventions shared by every call:
 *  - Qubit j is bit j of the amplitude index (little-endian, as in Qiskit,
 *    which the paper uses, Sec. V.A.1).  Segment 0 holds the lowest qubits;
 *    segments are contiguous blocks of qubits.
 *  - A state of m qubits is 2^m complex64 values, interleaved (re, im) float32,
 *    contiguous, in device memory.
 *  - Device pointers are plain addresses returned by hipMalloc (or a PyTorch
 *    tensor's data_ptr()).  The caller owns every device buffer it passes in.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls that take a stream only enqueue work and return; errors in kernels
 *    surface at the caller's next synchronisation.
 *  - Return value: CCUT_OK (0) or a negative CCUT_E* code; the message of the
 *    last failure on the calling thread is returned by ccut_last_error().
 *    No call aborts the process.
 */
#ifndef CCUT_H_
#define CCUT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ limits */
#define CCUT_MAX_SEG 8          /* segments per plan */
#define CCUT_MAX_Q 35           /* 2^35 complex64 = 256 GiB, the largest state one GPU holds */
#define CCUT_MAX_PLAN_Q 60      /* a plan's q when no merged state is formed (expectation values);
                                   every segment still holds at most CCUT_MAX_Q qubits */
#define CCUT_MAX_CUTS_PER_SEG 16 /* c_i <= 16: at most 65536 variants per segment */
#define CCUT_MAX_EXPECT_CUTS 12  /* c_i <= 12 for ccut_expectation_pauli (4096 x 4096 matrix per segment) */

/* ------------------------------------------------------------------ status */
#define CCUT_OK 0
#define CCUT_EINVAL (-1)        /* bad argument (q, sizes, gate kind, qubit index, NULL) */
#define CCUT_EUNCUTTABLE (-2)   /* a two-qubit gate joins two non-adjacent segments */
#define CCUT_ENOSPC (-3)        /* a caller buffer is smaller than required */
#define CCUT_ENOMEM (-4)        /* host or device allocation failed */
#define CCUT_EHIP (-5)          /* a HIP runtime call failed */
#define CCUT_EUNSUPPORTED (-6)  /* valid request this library does not implement */

/* ------------------------------------------------------------------ gates */
enum {
  CCUT_GATE_H = 0, CCUT_GATE_X = 1, CCUT_GATE_Y = 2, CCUT_GATE_Z = 3,
  CCUT_GATE_S = 4, CCUT_GATE_SDG = 5, CCUT_GATE_T = 6, CCUT_GATE_TDG = 7,
  CCUT_GATE_RX = 8,   /* exp(-i p0 X / 2) */
  CCUT_GATE_RY = 9,   /* exp(-i p0 Y / 2) */
  CCUT_GATE_RZ = 10,  /* exp(-i p0 Z / 2) */
  CCUT_GATE_RYRZ = 11,/* Ry(p0) . Rz(p1): Rz acts first */
  CCUT_GATE_CZ = 16,  /* symmetric in q0, q1 */
  CCUT_GATE_CX = 17,  /* q0 = control, q1 = target */
  /* Schmidt-rank-4 (and rank-2 Pauli-rotation) two-qubit gates, all symmetric
     in q0, q1; each is exp(-i/2 (tx XX + ty YY + tz ZZ)) up to a phase: */
  CCUT_GATE_SWAP = 18,  /* e^{i pi/4} exp(-i pi/4 (XX + YY + ZZ)) */
  CCUT_GATE_ISWAP = 19, /* |01> -> i|10>, |10> -> i|01>: exp(+i pi/4 (XX + YY)) */
  CCUT_GATE_RXX = 20,   /* exp(-i p0 XX / 2) */
  CCUT_GATE_RYY = 21,   /* exp(-i p0 YY / 2) */
  CCUT_GATE_RZZ = 22    /* exp(-i p0 ZZ / 2) */
};

/* One gate.  Single-qubit kinds ignore q1 (set it to -1); 32 bytes. */
typedef struct ccut_gate {
  int32_t kind;
  int32_t q0;
  int32_t q1;
  int32_t reserved; /* must be 0 */
  double p0;
  double p1;
} ccut_gate_t;

/* --------------------------------------------------------------- the plan */
typedef struct ccut_plan ccut_plan_t; /* opaque, owned by the library */

typedef struct ccut_plan_info {
  int32_t q;                           /* total qubits */
  int32_t n_seg;                       /* n */
  int32_t c_total;                     /* cut gates */
  int32_t n_gates;                     /* gates in the input circuit */
  int32_t seg_size[CCUT_MAX_SEG];      /* q_i */
  int32_t seg_offset[CCUT_MAX_SEG];    /* first qubit of segment i */
  int32_t c_seg[CCUT_MAX_SEG];         /* c_i: variant bits of segment i (one per adjacent
                                          rank-2 cut, two per rank-4 cut) */
  int32_t c_boundary[CCUT_MAX_SEG];    /* c_b: variant bits of the cuts between segments b and b+1 */
  int64_t n_sub;                       /* N_sub = sum_i 2^{c_i} = sum_i k^{cuts_i}  (Sec. III.A) */
  int64_t n_terms;                     /* 2^{sum_b c_b} global merge terms (Algorithm 3);
                                          INT64_MAX when that exceeds 2^62 */
  uint64_t seg_state_offset[CCUT_MAX_SEG]; /* byte offset of segment i's variant 0 in the arena */
  uint64_t state_bytes;                /* bytes of all subcircuit states */
  uint64_t arena_bytes;                /* the whole pipeline (simulation + merge workspace): size the arena to this */
  uint64_t psi_bytes;                  /* 8 * 2^q, the merged state */
  uint64_t sim_arena_bytes;            /* enough for ccut_simulate_subcircuits and ccut_expectation_pauli */
} ccut_plan_info_t;

typedef struct ccut_cut_info {
  int32_t gate_index; /* position in the input gate list (the first gate of a fused run) */
  int32_t kind;       /* gate kind (of the first gate of a fused run) */
  int32_t boundary;   /* b: the cut joins segments b and b+1 */
  int32_t q_low;      /* its qubit in segment b */
  int32_t q_high;     /* its qubit in segment b+1 */
  int32_t target_high;/* CX only: 1 if the target sits in segment b+1 */
  int32_t bit_low;    /* first bit of this cut in segment b's variant index */
  int32_t bit_high;   /* first bit of this cut in segment b+1's variant index */
  int32_t n_bits;     /* variant bits of the cut: 1 (rank 2), 2 (rank 4) */
  int32_t n_gates;    /* gates fused into this cut (1 unless a run of Pauli-rotation gates) */
} ccut_cut_info_t;

/*
 * Preprocessing, Algorithm 1 (Appendix B).  Scans the circuit for two-qubit
 * gates whose qubits lie in different segments, splits every segment's gate
 * list at them, and records, for each segment, one gate program with a
 * selectable S / S^dag slot per adjacent cut (the 2^{c_i} subcircuits of
 * Algorithm 1 are these programs with the slots fixed by the variant index;
 * they are never copied out).  Host-only; touches no GPU.
 *
 *   q          total qubits, 1..CCUT_MAX_PLAN_Q (ccut_merge_full_state needs
 *              q <= CCUT_MAX_Q); every segment at most CCUT_MAX_Q qubits
 *   gates      n_gates gates (host memory, read during the call only)
 *   n_seg      number of segments n, 1..CCUT_MAX_SEG
 *   seg_sizes  n_seg contiguous block sizes adding up to q, or NULL for
 *              floor(q/n) per block with the remainder on the last blocks
 *   plan_out   receives the plan; free it with ccut_plan_free
 *
 * Cut decompositions (Sec. II.A.2, Eqs. CZ and schmidt): CZ and CX use the
 * rank-2 form of Eq. (CZ), one variant bit (0: S term, 1: S^dag term).  The
 * other two-qubit kinds are cut through their operator-Schmidt decomposition:
 * every one of them is c * exp(-i/2 (tx XX + ty YY + tz ZZ)), which expands
 * exactly as sum_P c_P P (x) P over P in {I, X, Y, Z} (the Pauli products are
 * orthogonal, so this is the Schmidt form).  With two nonzero c_P (RXX, RYY,
 * RZZ alone) the cut has rank 2: one bit choosing between the two Paulis on
 * both sides.  Otherwise (SWAP, iSWAP, products) it has rank 4: two bits
 * (b0, b1) apply X^{b0} Z^{b1} on both sides with weights (c_I, c_X, c_Z,
 * -c_Y) for b0 + 2 b1 = 0..3 (Y = i X Z).  Consecutive Pauli-rotation gates
 * on the same cross-boundary pair, with nothing in between on either qubit,
 * commute and are fused into one cut: a general two-qubit unitary written as
 * local gates around RXX RYY RZZ costs one rank-4 cut.
 *
 * Cuts are numbered boundary by boundary (lowest boundary first) and in gate
 * order within a boundary; each takes n_bits consecutive variant bits.
 * Variant index r of segment i: its bits [0, c_{i-1}) select the terms of the
 * cuts on the boundary below it, the next c_i' bits those on the boundary
 * above it.
 * Arena layout: segment-major, then variant r, each state 2^{q_i} complex64
 * at seg_state_offset[i] + r * 8 * 2^{q_i} (256-byte aligned bases).
 *
 * Errors: CCUT_EINVAL (bad q, sizes, qubit or kind), CCUT_EUNCUTTABLE (a
 * two-qubit gate between non-adjacent segments), CCUT_EUNSUPPORTED (some
 * c_i > CCUT_MAX_CUTS_PER_SEG variant bits).
 */
int ccut_cut_plan(int32_t q, const ccut_gate_t* gates, int64_t n_gates, int32_t n_seg,
                  const int32_t* seg_sizes, ccut_plan_t** plan_out);

/*
 * Seeded input circuits (host-only; input data, not part of the method).
 *
 * ccut_brickwork: the random brickwork of the problem statement (Sec. IV: q
 * qubits, depth d, n contiguous segments, c_b cuts on boundary b).  Layer l
 * (0-based) applies RYRZ(theta, phi) to every qubit, then CZ(i, i + 1) for
 * i = l mod 2, l mod 2 + 2, ... except on the pairs that straddle a segment
 * boundary; boundary b instead gets exactly c_b CZ gates, at the end of layers
 * floor(j d / c_b), j = 0 .. c_b - 1, so c_total two-qubit gates cross the
 * boundaries.  Angles are 2 pi u with u = (x >> 11) 2^-53 and x the SplitMix64
 * (Steele, Lea and Flood 2014) stream of `seed`, drawn layer by layer, qubit
 * by qubit, theta before phi.
 *   seg_sizes: n sizes summing to q, or NULL for floor(q / n) with the
 *     remainder on the last segments.
 *   cuts_per_boundary: n - 1 counts summing to c_total, or NULL for an even
 *     split with the extras on the lower boundaries.  Each c_b <= d.
 *   out: caller-owned array of cap gates, or NULL to query the count.
 *   *n_out: the number of gates (also when out is NULL or too small).
 * ccut_staircase: the paper's own family (Fig. 1): H on every qubit, then
 * `copies` CX staircases CX(i, i + 1), i = 0 .. q - 2, each CX preceded by T on
 * its target (and, for i = 0, T on qubit 0) and followed by T on both qubits.
 * tx_layers > 0 adds the depth padding of Sec. V.D: that many (T, X) pairs on
 * qubit 0 before the first staircase and on qubit q - 1 after the last.
 * Errors: CCUT_EINVAL (shape, sizes, counts, c_b > d), CCUT_ENOSPC (cap too small).
 */
int ccut_brickwork(int32_t q, int32_t d, int32_t n_seg, int32_t c_total, const int32_t* seg_sizes,
                   const int32_t* cuts_per_boundary, uint64_t seed, ccut_gate_t* out, int64_t cap,
                   int64_t* n_out);
int ccut_staircase(int32_t q, int32_t copies, int32_t tx_layers, ccut_gate_t* out, int64_t cap, int64_t* n_out);

/* Sizes and counts of a plan (host-only). */
int ccut_plan_info(const ccut_plan_t* plan, ccut_plan_info_t* info);

/* Cut j (0 <= j < c_total) of a plan, in the plan's numbering (host-only). */
int ccut_plan_cut(const ccut_plan_t* plan, int32_t j, ccut_cut_info_t* out);

/*
 * Merge weight of cut term `bit` (0 or 1), Eq. (CZ): s_0 = 1/(1+i), s_1 = i/(1+i).
 * The weight of a global combination (alpha_m of Algorithm 3) is the product
 * over all cuts.  Writes (re, im) in float64 to out[0..1].  Host-only.
 */
int ccut_cut_weight(int32_t bit, double out[2]);

/*
 * Weights of the 2^{n_bits} terms of cut j (term t = its variant bits read as
 * an integer), (re, im) in float64 to w[2t], w[2t+1]; w holds 8 doubles.  For
 * CZ / CX these are s_0, s_1 of Eq. (CZ); for the other kinds the Schmidt
 * coefficients described at ccut_cut_plan.  The weight alpha_m of a global
 * combination is the product over all cuts.  Host-only.
 */
int ccut_plan_cut_terms(const ccut_plan_t* plan, int32_t j, double w[8]);

/* Frees a plan and its device tables.  NULL is ignored. */
void ccut_plan_free(ccut_plan_t* plan);

/*
 * Uploads the plan's device tables (gate programs, merge weights) on the
 * current device.  Part of T_pre.  Called implicitly by the first
 * simulate/merge call; call it explicitly before capturing those calls in a
 * HIP graph.  Synchronous.  Errors: CCUT_ENOMEM, CCUT_EHIP.
 */
int ccut_plan_prepare(ccut_plan_t* plan);

/*
 * Subcircuit simulation, Algorithm 2 (Appendix B): for every segment i and
 * variant r in [0, 2^{c_i}), psi_i^{(r)} = (segment i's gates with the cut
 * slots set by r) |0...0>, written to the arena at the plan's layout.
 * Complex64 states; the gate arithmetic follows ccut_plan_set_sim_precision.
 *
 *   d_arena      device buffer of at least info.arena_bytes bytes
 *   arena_bytes  its size
 * Errors: CCUT_ENOSPC (arena too small), CCUT_EINVAL, CCUT_EHIP.
 */
int ccut_simulate_subcircuits(ccut_plan_t* plan, void* d_arena, uint64_t arena_bytes, void* stream);

/* Merge precisions (Algorithm 3 arithmetic). */
enum {
  CCUT_PREC_AUTO = -1,   /* by term count: FP32 below K = 8 (or the autotuned threshold), else the
                            plan's split MFMA arithmetic: FP16X3 unless the autotuner found BF16X3
                            faster, or FP16X2 where ccut_plan_set_auto_precision asks for it */
  CCUT_PREC_FP32 = 0,    /* complex64 factors, float32 FMA accumulation (vector ALUs) */
  CCUT_PREC_BF16X3 = 1,  /* factors split hi + lo in bfloat16, hi.hi + hi.lo + lo.hi on MFMA, float32 accumulate */
  CCUT_PREC_FP16X3 = 2,  /* as BF16X3 with float16 halves and power-of-two pre-scaling */
  CCUT_PREC_BF16 = 3,    /* unsplit bfloat16 on MFMA: a low-accuracy control */
  CCUT_PREC_FP16X2 = 4   /* float16, only the high-qubit factor split: Lhi.R + Llo.R (R rounded once);
                            relative error of R <= 2^-11, 1 - F ~ 1e-7; explicit opt-in only */
};

/*
 * Merging, Algorithm 3 (Appendix B):
 *   Psi = sum over all info.n_terms cut-term combinations m of
 *         alpha_m  psi_{n-1}^{(r_{n-1}(m))} (x) ... (x) psi_0^{(r_0(m))},
 * alpha_m being the product of the per-cut term weights (Eq. CZ, or the
 * Schmidt coefficients).  For n >= 3 the sum is contracted boundary by
 * boundary (same result up to rounding).
 *
 *   d_arena    the arena filled by ccut_simulate_subcircuits for this plan; its
 *              workspace part (past info.sim_arena_bytes) is overwritten.  The
 *              merge weights are read from the table copy that call left in the
 *              arena (they are copied again if this plan's last simulation used
 *              another arena), so no other plan may use the arena in between
 *   d_psi      output, 2^q complex64 (psi_bytes >= info.psi_bytes); written once
 *   precision  one of CCUT_PREC_*
 * Errors: CCUT_ENOSPC, CCUT_EINVAL (unknown precision), CCUT_EHIP.
 */
int ccut_merge_full_state(ccut_plan_t* plan, void* d_arena, uint64_t arena_bytes, void* d_psi,
                          uint64_t psi_bytes, int32_t precision, void* stream);

/*
 * The uncut baseline T_orig (Sec. III.A): the whole circuit applied gate by
 * gate to |0...0> of q qubits, written to d_psi (2^q complex64).  The gate
 * list is compiled on the host (compiled programs are cached by content) and
 * run as LDS-blocked passes over the state in HBM, with the default
 * (CCUT_SIM_FP16X3) gate arithmetic of the subcircuit simulation.
 * Errors: CCUT_EINVAL, CCUT_ENOSPC, CCUT_ENOMEM, CCUT_EHIP.
 */
int ccut_simulate_uncut(int32_t q, const ccut_gate_t* gates, int64_t n_gates, void* d_psi,
                        uint64_t psi_bytes, void* stream);

/*
 * Float64 diagnostics of a 2^q complex64 state d_psi against an optional
 * reference d_ref (NULL: reference terms are 0).  Cutting reproduces the uncut
 * state exactly up to rounding (Sec. III); these measure how closely.
 *   out[0] = |psi|^2, out[1] = |ref|^2, out[2] = Re <ref|psi>,
 *   out[3] = Im <ref|psi>, out[4] = max_x |psi[x] - ref[x]|.
 * `out` is host memory; the call synchronises `stream` before returning.
 * Errors: CCUT_EINVAL, CCUT_EHIP.
 */
int ccut_norm_fidelity(const void* d_psi, const void* d_ref, int32_t q, double out[5], void* stream);

/*
 * Allocation-free variant of ccut_norm_fidelity, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same kernels and the same five results
 * in the same order as ccut_norm_fidelity, written to DEVICE memory d_out
 * (5 doubles, caller-owned, 8-byte aligned) instead of host memory.  The call
 * enqueues on `stream` and returns without synchronising or copying
 * to the host.  It calls no hipMalloc/hipFree: the per-block partials live in
 * a fixed device array of 1024 x 5 doubles (40 KiB) inside the library, one
 * copy per device, held until the process ends and looked up on the first call
 * on each device.  That covers every q <= CCUT_MAX_Q; larger q is rejected
 * with CCUT_EINVAL.  The array keeps the last call's partials; every partial a
 * call reads is written by that same call.  Calls that overlap on one device
 * (two streams, or two host threads without ordering between their streams)
 * share that array and race: order them on one stream.
 * Errors: CCUT_EINVAL (NULL pointer, q out of range), CCUT_EHIP.
 */
int ccut_norm_fidelity_noalloc(const void* d_psi, const void* d_ref, int32_t q, double* d_out, void* stream);

/*
 * Expectation value of a Pauli string on the cut state, from the subcircuit
 * states alone (the setting the paper's closing section names, Sec. VI: no
 * O(2^q) merge and no 2^q buffer).  With O = P_{n-1} x ... x P_0 split by the
 * segments, <Psi|O|Psi> = sum_{b,b'} conj(alpha_b) alpha_b' prod_i G_i[r_i(b)][r_i(b')]
 * where G_i[r][r'] = <psi_i^{(r)}| P_i |psi_i^{(r')}> is formed on the GPU
 * (float32 products, float64 sums) and the sum over the cut bits is contracted
 * boundary by boundary in float64 on the host.  Work: sum_i 4^{c_i} 2^{q_i}.
 *
 *   d_arena    the arena after ccut_simulate_subcircuits (read only)
 *   pauli      q characters from "IXYZ"; character j acts on qubit j
 *   d_work     device workspace of ccut_expectation_work_bytes() bytes
 *   out        host: real and imaginary part (the latter ~0 for a Pauli string)
 * Synchronises `stream`.  Errors: CCUT_EINVAL (label), CCUT_ENOSPC,
 * CCUT_EUNSUPPORTED (more than CCUT_MAX_EXPECT_CUTS cuts on a segment: its
 * 4^{c_i} matrix entries would exceed one launch grid), CCUT_EHIP.
 */
int ccut_expectation_work_bytes(const ccut_plan_t* plan, uint64_t* bytes);
int ccut_expectation_pauli(ccut_plan_t* plan, const void* d_arena, uint64_t arena_bytes, const char* pauli,
                           void* d_work, uint64_t work_bytes, double out[2], void* stream);

/* ------------------------------------------------- launches, graphs, tuning */
/*
 * Launch configuration of a plan's subcircuit simulation (the batched
 * subcircuit stage of Algorithm 2):
 *   threads      workgroup size of the simulation kernel: 256, 512 or 1024
 *   grid_cap     0: one workgroup per amplitude block; > 0: a persistent grid of
 *                at most grid_cap workgroups looping over all blocks of all variants
 *   per_variant  0: one launch covers every variant of every segment (per pass);
 *                1: one launch per (segment, variant), the unbatched reference
 *   mfma_min_terms  CCUT_PREC_AUTO merges on MFMA (ccut_plan_get_auto_precision) from this term
 *                count K (-1: library default 8)
 * Results do not depend on the configuration.  ccut_plan_get_launch returns
 * (threads, grid_cap, per_variant, mfma_min_terms).  Host-only.
 */
int ccut_plan_set_launch(ccut_plan_t* plan, int32_t threads, int32_t grid_cap, int32_t per_variant,
                         int32_t mfma_min_terms);
int ccut_plan_get_launch(const ccut_plan_t* plan, int32_t out[4]);

/*
 * Shape of a plan's compiled simulation programs (host-only): out[0] pass
 * descriptors, [1] register stages, [2] device op records (a group of 2x2
 * gates on distinct register positions is one header plus one record per
 * position), [3] dense ops (2x2 and CX), [4] diagonal ops, [5] fused register-level ops of all segments,
 * [6] simulation launches, [7] (segment, variant, pass) jobs.  Counts cover
 * every segment once (variants share their segment's program).
 */
int ccut_plan_stats(const ccut_plan_t* plan, int64_t out[8]);

/*
 * Work the plan's simulation launches execute (host-only), summed over every
 * job of the current schedule (flat or prefix tree, at the current block size):
 * out[0] dense 2x2 gate applications x amplitudes, out[1] diagonal ones (phases,
 * scalars), out[2] permutation and sign ops (CX, CZ), out[3] amplitudes moved
 * between HBM (or L2) and LDS (a pass that starts from |0...0> only writes),
 * out[4] the dense gate applications x amplitudes of the flat schedule (every
 * fused gate of a segment on every variant), for comparison.
 */
int ccut_plan_work(const ccut_plan_t* plan, double out[5]);

/*
 * Variant and grid of the MFMA merge GEMM.  epilogue 0..3 are tiled kernels:
 * bit 0 set transposes 16-row slabs through LDS into 16-byte row stores
 * (clear: each lane stores its accumulators directly); bit 1 set uses 64 x 256
 * tiles with 32 rows per wavefront (clear: 128 x 256 tiles, 64 rows per
 * wavefront).  epilogue 4 is the R-stationary kernel: one 16-wavefront
 * workgroup per CU keeps a 128-column strip of the low-qubit factor (all
 * terms, hi and lo) in LDS and sweeps all rows of its strip; it covers up to
 * K = 64 terms per stage and runs larger stages as epilogue 1.  epilogue 5 is
 * the LDS-staged kernel for many terms: one 8-wavefront workgroup per CU loops
 * over 256-row x 256-column tiles, copying each MFMA step's fragments of both
 * factors from L2 straight into LDS once per tile (four steps ahead, four
 * buffers) for all its wavefronts; stages with fewer than 256 rows or fewer than
 * 32 terms run as epilogue 1.  epilogue 6 is the column-stationary kernel: one
 * 8-wavefront workgroup per CU owns a 128-column strip; four wavefronts keep two
 * 32-column blocks each of the low-qubit factor in registers and compute, four
 * fetch the high-qubit factor's fragments into LDS and store each 32-row tile
 * through LDS as whole 1 KiB row segments; it covers up to K = 64 terms per stage
 * and runs larger stages as epilogue 1.
 * grid_cap 0 launches one workgroup per tile, > 0 a persistent grid of at most
 * grid_cap workgroups looping over tiles (ignored by epilogues 4 to 6, which size
 * their own grids).  Results do not depend on either.  A new plan starts at
 * epilogue 6 when no stage has more than 64 terms, else at 5.
 * Host-only.  Errors: CCUT_EINVAL.
 */
int ccut_plan_set_merge(ccut_plan_t* plan, int32_t epilogue, int32_t grid_cap);
/* The current (epilogue, grid_cap) of a plan (host-only). */
int ccut_plan_get_merge(const ccut_plan_t* plan, int32_t out[2]);

/*
 * The MFMA arithmetic CCUT_PREC_AUTO uses for merge stages at or above the
 * plan's term threshold: CCUT_PREC_FP16X3 (default), CCUT_PREC_BF16X3, or
 * CCUT_PREC_FP16X2 as an explicit opt-in (its max-abs error is larger: the
 * low-qubit factor is rounded once to float16).  ccut_autotune sets it to the
 * faster of the two fully split arithmetics.  Host-only.  Errors: CCUT_EINVAL.
 */
int ccut_plan_set_auto_precision(ccut_plan_t* plan, int32_t precision);
int ccut_plan_get_auto_precision(const ccut_plan_t* plan, int32_t* out);

/* Gate arithmetic of the state-vector simulation (Algorithm 2 and the uncut baseline). */
enum {
  CCUT_SIM_FP32 = 0,    /* every gate in float32 on the vector ALUs */
  CCUT_SIM_FP16X3 = 1   /* default: each register-stage group of single-qubit gates (one per
                           register qubit, a 16x16 complex Kronecker product) as split-float16
                           MFMA, hi.hi + hi.lo + lo.hi with float32 accumulation on a state
                           scaled by 2^14; relative error per group ~1e-6; other ops float32 */
};

/*
 * Gate arithmetic of a plan's subcircuit simulation (CCUT_SIM_*).  Host-only.
 * Errors: CCUT_EINVAL.
 */
int ccut_plan_set_sim_precision(ccut_plan_t* plan, int32_t precision);
/* The plan's current CCUT_SIM_* value (host-only). */
int ccut_plan_get_sim_precision(const ccut_plan_t* plan, int32_t* out);

/*
 * LDS block size of the subcircuit simulation (Algorithm 2): blocks of 2^bits
 * amplitudes, bits in (4, 14]; 0 restores the automatic choice (the largest
 * size whose first launch has a workgroup per compute unit, not below 2^12).
 * A segment with more qubits than bits is simulated in several passes over
 * its state in HBM; smaller blocks trade passes for parallelism when there
 * are fewer variants than compute units.  A pass whose op headers and stage
 * heads would not fit in LDS beside its block (deep circuits in large blocks)
 * is split into consecutive passes over the same qubits.  Reschedules the plan's programs
 * (host-only) and may enlarge ccut_plan_info().arena_bytes: query it again
 * before sizing an arena.  Results agree to float32 rounding across sizes.
 * Errors: CCUT_EINVAL.
 */
int ccut_plan_set_block_bits(ccut_plan_t* plan, int32_t bits);
/* The block bits the plan's simulation tables are built for (host-only). */
int ccut_plan_get_block_bits(const ccut_plan_t* plan, int32_t* out);

/*
 * Prefix sharing in the subcircuit simulation (Algorithm 2 re-simulates the
 * gates before a cut for every variant).  mode 1: each segment program is cut
 * before each of its slotted ops (in program order); level l holds the 2^l
 * states of the first l slot choices and level l + 1 applies the next chunk to
 * each, once per choice of its slot, so the gates before a slot run once per
 * prefix instead of once per variant.  One launch per level and LDS pass;
 * levels below the last use a scratch region of the arena.  mode 0: every
 * variant from |0...0> in one launch per pass.  mode -1 (default): on when the
 * variants hold at least 2^23 amplitudes in all.  Results agree to float32
 * rounding.  Host-only; reschedules the plan.  Errors: CCUT_EINVAL.
 */
int ccut_plan_set_prefix_sharing(ccut_plan_t* plan, int32_t mode);
/* 1 if the plan's tables use prefix sharing, else 0 (host-only). */
int ccut_plan_get_prefix_sharing(const ccut_plan_t* plan, int32_t* out);
/*
 * First level of the prefix-sharing tree (default 0).  With level L, segment i's
 * first min(L, c_i) slots are not shared: its 2^min(L, c_i) level-L states run
 * the program up to slot L from |0...0> in one launch, and the tree branches
 * from there.  The early levels hold few states and leave most of the device
 * idle; starting later trades them for some repeated gates.  L >= c_i is the
 * flat simulation.  Host-only; reschedules the plan.  Errors: CCUT_EINVAL
 * (L outside [0, CCUT_MAX_CUTS_PER_SEG]).
 */
int ccut_plan_set_prefix_start(ccut_plan_t* plan, int32_t level);
int ccut_plan_get_prefix_start(const ccut_plan_t* plan, int32_t* out);

/*
 * Gate fusion in the register stages of the subcircuit simulation (the gates of
 * Algorithm 2, applied in the same order): on = 1 folds, inside each stage, the
 * runs of single-qubit gates, diagonal phases, CZ pairs and CX gates that act on
 * the stage's four register qubits alone into one 16x16 matrix, applied as one
 * split-float16 MFMA product, and applies the stage's CZ pairs between qubits
 * outside its register set once, at its end (they commute with everything the
 * stage does).  The matrices are composed (float64) on the device by every
 * ccut_simulate_subcircuits call, which costs more than it saves when a plan is
 * simulated once; off = 0 is the default.  The uncut baseline always fuses: its
 * programs are cached and their matrices built once.  Results agree to float32
 * rounding.  Host-only; reschedules the plan.  Errors: CCUT_EINVAL.
 */
int ccut_plan_set_fusion(ccut_plan_t* plan, int32_t on);
int ccut_plan_get_fusion(const ccut_plan_t* plan, int32_t* out);

/*
 * Autotuner: times the simulation kernel over prefix sharing off / on (tree
 * from level 0, 2, 3, 4, c - 2 and c - 1, c the largest c_i) x LDS
 * block sizes (whole segment, 2 and 4 blocks per state; sizes whose tables do
 * not fit arena_bytes are skipped) x workgroup sizes x persistent grid sizes,
 * and the merge with the
 * float32 kernel against the fully split MFMA GEMM (FP16X3 and BF16X3) over its
 * variants and grids (median of `reps` runs, HIP events on `stream`; every merge run follows
 * an untimed simulation, as in the pipeline, and each GEMM candidate is timed in
 * a forward and a backward sweep, median of max(reps, 7) runs each, keeping the
 * better median, since short merges see clock drift; the plan's current split
 * arithmetic, GEMM variant and grid are kept unless another is more than 2 % faster;
 * BF16X3, the less accurate split, is taken only if more than 2 % faster than FP16X3),
 * applies the fastest (AUTO then merges in the chosen split arithmetic)
 * to the plan and records it in a process-wide cache keyed by (architecture,
 * plan shape); later plans of the same shape start from it (their tables, and so
 * their info.arena_bytes, can be larger than the tuning plan's: size an arena
 * from the plan that will use it).  The block size and
 * prefix-sharing mode regroup the gates, so a tuned plan's states agree with the
 * untuned ones to float32 rounding (not bit for bit).  Overwrites the arena and
 * d_psi.  *best_ms (nullable) receives the tuned simulation + merge time.
 * ccut_autotune_save / _load write and read the cache as text (one
 * "key threads grid_cap mfma_min_terms epilogue merge_grid block_bits prefix
 * mfma_mode" line per entry; prefix 0 = off, 1 + L = on with the tree from level
 * L; mfma_mode is AUTO's split arithmetic and may be absent, meaning FP16X3).
 * Errors: CCUT_EINVAL, CCUT_ENOSPC, CCUT_EHIP.
 */
int ccut_autotune(ccut_plan_t* plan, void* d_arena, uint64_t arena_bytes, void* d_psi, uint64_t psi_bytes,
                  int32_t reps, void* stream, double* best_ms);
int ccut_autotune_save(const char* path);
int ccut_autotune_load(const char* path);

/*
 * HIP graph of a plan's whole device pipeline (subcircuit simulation, then
 * merge at `precision`; Algorithms 2 and 3 as one replayable unit) captured on
 * `stream` (must not be the default stream).  The graph owns a device copy of
 * the plan's tables, made at capture, so replays copy nothing from the host;
 * the plan can be freed once the graph exists.  The arena and d_psi addresses
 * are baked into the graph and must stay valid.  ccut_graph_launch replays it
 * on any stream.  Do not use the plan from another thread while it is captured.
 * Errors: CCUT_EINVAL, CCUT_ENOSPC, CCUT_ENOMEM, CCUT_EHIP.
 */
typedef struct ccut_graph ccut_graph_t;
int ccut_graph_create(ccut_plan_t* plan, void* d_arena, uint64_t arena_bytes, void* d_psi, uint64_t psi_bytes,
                      int32_t precision, void* stream, ccut_graph_t** out);
int ccut_graph_launch(ccut_graph_t* graph, void* stream);
void ccut_graph_free(ccut_graph_t* graph);

/*
 * Points a graph at another plan of the same launch layout (same circuit shape,
 * segment sizes, cut positions and fused program lengths, launch configuration
 * and table layout; typically the same circuit family with other angles):
 * enqueues on `stream` a copy of that plan's tables into the graph's table copy.
 * Replays on `stream` after this call compute the new plan's pipeline; a replay
 * enqueued earlier on `stream` still reads the old tables (stream order), so
 * rebind and launch on one stream.  The plan may be freed after the call.
 * Errors: CCUT_EINVAL (NULL, other device, or a different launch layout),
 * CCUT_EHIP.
 */
int ccut_graph_rebind(ccut_graph_t* graph, const ccut_plan_t* plan, void* stream);

/* ------------------------------------------------------------ cost model */
/*
 * Closed-form subcircuit-stage threshold of Sec. IV for equal partitioning
 * into n segments (k = 2): c_total < *bound, with *bound = q/2 for n = 2
 * (Eq. threshold_n2) and q (n-1)^2/(2n) + (n-1) log2(n/(n-2))/2 for n >= 3
 * (Eq. threshold_nge3, Table II).  Host-only.  Errors: CCUT_EINVAL.
 */
int ccut_threshold_ctotal(int32_t q, int32_t n, double* bound);

/*
 * log2 margin of Eq. (speedup_depth_free), N_sub / n < 2^{q (1 - 1/n)}, with
 * N_sub = sum_i 2^{c_i} counted exactly from n-1 cut counts per boundary:
 * q (1 - 1/n) - log2(N_sub / n).  Positive: the subcircuit stage beats the
 * uncut simulation.  Host-only.  Errors: CCUT_EINVAL.
 */
int ccut_speedup_margin(int32_t q, int32_t n, const int32_t* cuts_per_boundary, double* margin);

/*
 * The learned cost model (not part of the paper): an 8-64-64-3 tanh MLP,
 * CCUT_MLP_PARAMS float32 parameters laid out W1[8][64], b1[64], W2[64][64],
 * b2[64], W3[64][3], b3[3], mapping features of (q, d, n, c_total) to
 * ln T_pre, ln T_sub, ln T_merge in seconds (an uncut run is the row n = 1,
 * c_total = 0 with T_orig in the T_sub slot).
 *
 * ccut_cost_features: the 8 input features (host), all functions of
 * (q, d, n, c_total) for equal blocks and cuts spread evenly over the n - 1
 * boundaries: (q - 24) / 8, log2 d - log2 20, n - 3, (c_total - 4) / 4, then
 * the cost terms of Table I: (log2 N_sub - 6) / 4 with N_sub = sum_i 2^{c_i},
 * (q_max - 12) / 4 with q_max = ceil(q / n), (log2 N_sub + q_max + log2 d - 24) / 6
 * (subcircuit stage, N_sub 2^{q_max} d) and (c_total + q - 30) / 6 (merge,
 * 2^{c_total} terms over 2^q amplitudes).  Uncut: n = 1, c_total = 0,
 * N_sub = 1, q_max = q.
 * ccut_mlp_predict: d_y[rows][3] = net(d_x[rows][8]) on the device.
 * ccut_mlp_grad: mean-squared-error loss against d_t[rows][3] (written to
 *   host *loss) and its gradient d_grad[CCUT_MLP_PARAMS]; synchronous.
 * ccut_mlp_train: `epochs` full-batch Adam steps (lr, betas 0.9 / 0.999,
 *   eps 1e-8) updating d_params in place; the per-epoch losses go to host
 *   `losses` (epochs floats, or NULL).  Work buffer: ccut_mlp_work_bytes.
 *   Synchronous.  A non-default stream lets training replay captured HIP
 *   graphs of 50 epochs.
 * All d_ pointers are device memory owned by the caller.
 * Errors: CCUT_EINVAL, CCUT_ENOSPC (work buffer), CCUT_EHIP.
 */
#define CCUT_MLP_PARAMS 4931
int ccut_cost_features(int32_t q, int32_t d, int32_t n, int32_t c_total, float out[8]);
int ccut_mlp_work_bytes(int64_t rows, int32_t epochs, uint64_t* bytes);
int ccut_mlp_predict(const float* d_params, const float* d_x, int64_t rows, float* d_y, void* stream);
int ccut_mlp_grad(const float* d_params, const float* d_x, const float* d_t, int64_t rows, void* d_work,
                  uint64_t work_bytes, float* d_grad, float* loss, void* stream);
int ccut_mlp_train(float* d_params, const float* d_x, const float* d_t, int64_t rows, int32_t epochs, float lr,
                   void* d_work, uint64_t work_bytes, float* losses, void* stream);

/*
 * Whether and how to cut a circuit of q qubits, depth d and c_total cut
 * gates.  Candidates: no cut, and n = 2, 3, 4 equal segments with the cuts
 * spread evenly over the n-1 boundaries.
 *  - d_params == NULL: the closed-form rule of Sec. IV: the n whose
 *    Eq. (speedup_depth_free) margin is largest and positive, else no cut;
 *    *predicted_s = NaN.  Host-only.
 *  - otherwise: the learned model predicts each candidate's wall clock
 *    (T_pre + T_sub + T_merge, or T_orig) and the smallest wins, except that
 *    the closed-form choice is kept unless the winner is predicted faster than
 *    it by more than the fraction `margin` (0 <= margin < 1; 0: plain argmin).
 *    *predicted_s is the chosen candidate's prediction.  If budget_s > 0 and
 *    it exceeds the budget, *choice = -1 (infeasible).  Synchronises `stream`.
 * *choice: 0 = simulate uncut, n >= 2 = cut into n segments, -1 = infeasible.
 * Errors: CCUT_EINVAL, CCUT_EHIP.
 */
int ccut_decide(int32_t q, int32_t d, int32_t c_total, const float* d_params, double budget_s, double margin,
                int32_t* choice, double* predicted_s, void* stream);

/*
 * Kernel timing.  While enabled, every kernel this library launches is
 * bracketed by HIP events recorded on the stream it runs on (a few
 * microseconds of overhead per launch).  ccut_profile_read waits for the
 * recorded events, folds them into per-family totals and returns, for kernel
 * family `kernel` (0 <= kernel < CCUT_PROF_KERNELS), the number of launches
 * and their summed device milliseconds since the last reset, plus the family
 * name ("sim", "merge_f32", "split", "tables", "merge_gemm", "reduce",
 * "mlp", "expect"; a static string, pass NULL to skip).  "split" is the
 * packing of both merge GEMM operands (one launch per GEMM merge stage);
 * "tables" the device copies of a plan's op and gate tables and the MFMA
 * group tables built from them.  Errors: CCUT_EINVAL, CCUT_EHIP.
 */
#define CCUT_PROF_KERNELS 8
int ccut_profile_enable(int32_t on);
int ccut_profile_read(int32_t kernel, int64_t* launches, double* total_ms, const char** name);
int ccut_profile_reset(void);
/* Families timed while enabled: bit k set times family k (default: all). */
int ccut_profile_mask(uint32_t mask);

/* Message of the last failed call on this thread ("" if none). */
const char* ccut_last_error(void);

/* Library build identification string (static). */
const char* ccut_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CCUT_H_ */
