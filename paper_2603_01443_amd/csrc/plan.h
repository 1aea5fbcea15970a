// The cut plan: preprocessing output (Algorithm 1) plus its device tables.
#pragma once

#include <mutex>

#include "ccut_internal.h"

struct ccut_plan {
  struct Seg {
    int32_t q = 0, off = 0;       // size, first qubit
    int32_t c_lo = 0, c_hi = 0;   // cuts on the boundary below / above
    int32_t c = 0;                // c_i
    uint64_t arena_off = 0;       // bytes
    ccut::Program prog;
    std::vector<ccut::Pass> passes;
    // prefix sharing: the program cut before each slotted op (level l >= 1 starts at the
    // op of slot chunk_slot[l - 1]); chunk_passes[l] are the LDS passes of chunk l
    std::vector<std::vector<ccut::Pass>> chunk_passes;
    std::vector<int32_t> chunk_slot;
    uint64_t tree_off = 0;  // bytes: ping-pong scratch of the prefix levels 0..c-1
  };
  int32_t q = 0, n_seg = 0, n_gates = 0;
  std::vector<Seg> segs;
  std::vector<ccut_cut_info_t> cuts;
  // How each cut is decomposed (Eq. CZ for CZ / CX, the Pauli form of Eq. schmidt
  // for the Pauli-rotation kinds) and the weights of its 2^{n_bits} terms.
  struct CutTerms {
    int form = 0;        // 0: S / S^dag (Eq. CZ), 1: one bit choosing Pauli pa or pb, 2: X^{b0} Z^{b1}
    int pa = 0, pb = 0;  // form 1: the two Paulis (0 I, 1 X, 2 Y, 3 Z)
    ccut::cd w[4];       // term weights, term t = the cut's variant bits as an integer
  };
  std::vector<CutTerms> cut_terms;
  std::vector<std::vector<ccut::cd>> bw;  // per boundary: weight of each of its 2^{c_b} term combinations
  std::vector<int32_t> c_b;
  uint64_t state_bytes = 0, arena_bytes = 0, psi_bytes = 0;
  uint64_t temp_off[2] = {0, 0};  // ping / pong temp regions of the chain merge (bytes)
  uint64_t temp_bytes[2] = {0, 0};
  bool merge_ok = true;           // the merged 2^q state fits (q <= CCUT_MAX_Q)
  uint64_t sim_bytes = 0;         // arena prefix used by the simulation (states, scratch, tables)
  uint64_t split_off = 0, split_bytes = 0;  // split-precision planes of the last merge stage
  std::vector<ccut::MergeStage> stages;
  std::vector<float> weights;     // complex64 merge weights, per stage

  // simulation launches: one per pass index, jobs for every (segment, variant)
  int bmax = ccut::PASS_MAX_B, low_bits = 4;  // bmax: block bits in use
  int block_bits = 0;                         // requested block bits, 0: automatic
  int prefix_mode = -1;                       // prefix sharing: 0 off, 1 on, -1 automatic
  int prefix_start = 0;                       // first tree level (the slots below it run flat)
  bool prefix_on = false;                     // in use by the current tables
  bool fuse = false;                          // register-stage gate fusion (ccut_plan_set_fusion)
  std::vector<ccut::PassDesc> pass_descs;
  std::vector<ccut::StageDesc> stage_descs;
  std::vector<ccut::KOp> kops;
  std::vector<ccut::GroupRef> grefs;  // MFMA operand tables of the register-stage groups
  std::vector<ccut::SimJob> jobs;
  // rec_cap: LDS room for the op headers and stage heads of its largest pass
  struct Launch { int job_begin, n_jobs, total_wg, rec_cap = 0; };
  std::vector<Launch> launches;

  // Packed table image (ops | passes | jobs | weights) and where it sits in the arena.
  std::vector<unsigned char> image;
  uint64_t img_ops = 0, img_passes = 0, img_stages = 0, img_jobs = 0, img_weights = 0, img_grefs = 0;
  uint64_t gtab_off = 0, gtab_reserve = 0;  // arena region of the MFMA group tables
  uint64_t tree_off = 0, tree_bytes = 0;    // arena region of the prefix-sharing scratch
  uint64_t tables_off = 0;  // arena byte offset of the table region
  uint64_t tables_reserve = 0;  // bytes reserved for it
  uint64_t total_arena = 0; // bytes the caller's arena must hold
  uint64_t image_gen = 0;   // bumped whenever the table image is rebuilt
  // arena (and image build) whose table region last received this plan's image
  const void* staged_arena = nullptr;
  uint64_t staged_gen = 0;

  // expectation values: pinned host copy of the per-segment matrices (grow-only,
  // freed with the plan); the mutex serialises calls that share it
  void* expect_host = nullptr;
  uint64_t expect_host_bytes = 0;
  std::mutex expect_mu;

  ccut::DeviceTables dev;   // plan-owned copy after ccut_plan_prepare (graph capture)
  std::vector<ccut::DeviceTables> retired;  // copies of earlier table builds (graphs may still use them)

  // launch configuration (ccut_plan_set_launch / ccut_autotune)
  int sim_threads = 1024;    // workgroup size of the simulation kernel
  int sim_grid_cap = 0;      // 0: one workgroup per block; > 0: persistent grid of this size
  int sim_per_variant = 0;   // 1: one launch per (segment, variant) instead of one per pass index
  int auto_mfma_min_k = -1;  // CCUT_PREC_AUTO threshold on K (-1: library default)
  int auto_mfma_mode = CCUT_PREC_FP16X3;  // CCUT_PREC_AUTO arithmetic at and above that K
  int merge_epilogue = 1;    // MFMA merge GEMM variant (see merge_mfma.h)
  int merge_grid_cap = 0;    // MFMA merge: 0 one workgroup per tile, > 0 persistent grid
  int sim_precision = CCUT_SIM_FP16X3;  // register-stage gate groups: split-float16 MFMA or float32 VALU
};

namespace ccut {
constexpr int AUTO_TARGET_WG = 256;      // workgroups the first simulation launch should reach (one per CU)
constexpr int AUTO_MIN_BLOCK_BITS = 12;  // smallest block the automatic choice goes down to
constexpr int AUTO_PREFIX_LOG2_AMPS = 23;  // automatic prefix sharing from 2^23 variant amplitudes on
bool auto_prefix(const ccut_plan* P);
uint64_t align256(uint64_t x);
int auto_block_bits(const ccut_plan* P);
// (Re)schedules the simulation at the plan's block size and repacks its tables.
int build_sim_tables(ccut_plan* P, bool first);
// Appends a pass to the device tables; returns its PassDesc index (fuse: see stage_kops).
int append_pass(const Pass& p, int nq, std::vector<PassDesc>& descs, std::vector<StageDesc>& stages,
                std::vector<KOp>& kops, std::vector<GroupRef>& grefs, bool fuse);
int gate_matrix(const ccut_gate_t& g, cd m[4]);
void release_device(DeviceTables& t);
// Copies a table image to a new device allocation (synchronous).
int upload_tables(DeviceTables& t, const std::vector<unsigned char>& img, uint64_t o_ops, uint64_t o_pass,
                  uint64_t o_stage, uint64_t o_jobs, uint64_t o_w, uint64_t o_grefs);
// Packs the tables into one image with 256-byte aligned sections.
void pack_image(ccut_plan* P);
// Applies a cached autotuned launch configuration to a new plan, if any.
void apply_tuned(ccut_plan* P);
// Enqueues a copy of `bytes` host bytes to device memory `dst` through a pinned staging ring.
int staged_copy(void* dst, const void* src, uint64_t bytes, hipStream_t s);
}  // namespace ccut
