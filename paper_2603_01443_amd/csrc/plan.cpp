// Preprocessing (Algorithm 1, Appendix B): find the cut gates, build one gate
// program per segment with an S / S^dag slot per adjacent cut, size the arena,
// and lay out the merge stages of Algorithm 3.
#include "plan.h"
#include "merge_mfma.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>

namespace ccut {

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

int append_pass(const Pass& p, int nq, std::vector<PassDesc>& descs, std::vector<StageDesc>& stages,
                std::vector<KOp>& kops, std::vector<GroupRef>& grefs, bool fuse) {
  PassDesc d;
  std::memset(&d, 0, sizeof(d));
  d.b = (int32_t)p.group.size();
  d.nq = nq;
  d.op_begin = (int32_t)kops.size();
  d.op_count = (int32_t)p.kops.size();
  d.init = p.init ? 1 : 0;
  d.from_src = p.from_src ? 1 : 0;
  d.n_blocks = 1 << (nq - d.b);
  std::vector<uint8_t> in(nq, 0);
  for (int j = 0; j < d.b; ++j) {
    d.group[j] = p.group[j];
    in[p.group[j]] = 1;
  }
  int f = 0;
  for (int t = 0; t < nq; ++t)
    if (!in[t]) d.fixed[f++] = t;
  if (d.b >= STAGE_MIN_B) {
    // register stages carry their own (stage-level) op ranges
    std::vector<StageDesc> st;
    std::vector<KOp> sk;
    stage_kops(p.kops, d.b, st, sk, fuse);
    const int32_t base = (int32_t)kops.size();
    for (StageDesc& s : st) s.op_begin += base;
    d.stage_begin = (int32_t)stages.size();
    d.stage_count = (int32_t)st.size();
    d.op_begin = base;
    d.op_count = (int32_t)sk.size();
    stages.insert(stages.end(), st.begin(), st.end());
    kops.insert(kops.end(), sk.begin(), sk.end());
    // one MFMA operand table per group (or fused run) and choice of its slots; the
    // records inside a fused run need none (the float32 path reads their matrices)
    for (size_t i = base; i < kops.size(); ++i) {
      KOp& g = kops[i];
      if (g.type != KOP_GROUP && g.type != KOP_FUSED) continue;
      const int nslot = (g.b >= 0) + (g.slot >= 0) + (g.cond >= 0) + (g.nterms >= 0);
      g.pad[0] = (int32_t)grefs.size();
      g.pad[1] = nslot;
      for (int sel = 0; sel < (1 << nslot); ++sel) grefs.push_back(GroupRef{(int32_t)i, sel});
      i += g.type == KOP_GROUP ? REG_BITS : g.a;
    }
  } else {
    kops.insert(kops.end(), p.kops.begin(), p.kops.end());
  }
  descs.push_back(d);
  return (int)descs.size() - 1;
}


// Largest block size whose first simulation launch still gives every compute
// unit of the device a workgroup; never below 2^12 amplitudes per block.
int auto_block_bits(const ccut_plan* P) {
  int b = PASS_MAX_B;
  for (; b > AUTO_MIN_BLOCK_BITS; --b) {
    int64_t wg = 0;
    for (const auto& S : P->segs) wg += ((int64_t)1 << S.c) << std::max(0, S.q - b);
    if (wg >= AUTO_TARGET_WG) break;
  }
  return b;
}

// Prefix sharing pays once the variants carry enough work to fill the device by
// themselves (then the stage is throughput-bound and shared prefixes are saved
// work); below that the sequential gate chain of one state sets the time.
bool auto_prefix(const ccut_plan* P) {
  uint64_t amps = 0;
  bool any = false;
  for (const auto& S : P->segs) {
    amps += ((uint64_t)1 << S.c) << S.q;
    any = any || S.c > 0;
  }
  return any && amps >= ((uint64_t)1 << AUTO_PREFIX_LOG2_AMPS);
}

// Prefix sharing (a tree over the slots in program order): level l holds the 2^l
// states of the first l slot choices; level l + 1 applies chunk l + 1 (which
// starts at slot l + 1's op) to each of them, once per choice of that slot.
// The tree starts at level L = min(prefix_start, c): its 2^L states run the
// program up to slot L from |0...0> (the early levels hold too few states to
// fill the device, so they are traded for some repeated work).  Levels below c
// live in a ping-pong scratch, level c is the arena layout.
int build_tree_launches(ccut_plan* P) {
  const int n_seg = P->n_seg;
  int max_c = 0;
  for (auto& S : P->segs) {
    S.chunk_passes.clear();
    S.chunk_slot.clear();
    std::vector<int> pos;
    for (int o = 0; o < (int)S.prog.ops.size(); ++o)
      if (S.prog.ops[o].slot >= 0) {
        pos.push_back(o);
        S.chunk_slot.push_back(S.prog.ops[o].slot);
      }
    if ((int)pos.size() != S.c) return fail(CCUT_EINVAL, "segment program has %zu slotted ops for %d cuts",
                                            pos.size(), S.c);
    const int L0 = std::min(P->prefix_start, S.c);
    S.chunk_passes.resize(S.c + 1);
    for (int l = L0; l <= S.c; ++l) {
      Program chunk;
      chunk.nq = S.prog.nq;
      const int begin = l == L0 ? 0 : pos[l - 1];
      const int end = l < S.c ? pos[l] : (int)S.prog.ops.size();
      chunk.ops.assign(S.prog.ops.begin() + begin, S.prog.ops.begin() + end);
      if (int rc = schedule_passes(chunk, P->bmax, P->low_bits, S.chunk_passes[l], l == L0, P->fuse)) return rc;
    }
    max_c = std::max(max_c, S.c);
  }
  for (int l = 0; l <= max_c; ++l) {
    size_t max_passes = 0;
    for (auto& S : P->segs)
      if (l <= S.c) max_passes = std::max(max_passes, S.chunk_passes[l].size());
    for (size_t p = 0; p < max_passes; ++p) {
      ccut_plan::Launch L{(int)P->jobs.size(), 0, 0};
      std::vector<int> order;
      for (int i = 0; i < n_seg; ++i)
        if (l <= P->segs[i].c && l >= std::min(P->prefix_start, P->segs[i].c) &&
            P->segs[i].chunk_passes[l].size() > p)
          order.push_back(i);
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return P->segs[a].q > P->segs[b].q; });
      for (int i : order) {
        auto& S = P->segs[i];
        int pid = append_pass(S.chunk_passes[l][p], S.q, P->pass_descs, P->stage_descs, P->kops, P->grefs, P->fuse);
        int nb = P->pass_descs[pid].n_blocks;
        const uint64_t half = S.c > 0 ? ((uint64_t)1 << (S.c - 1)) << S.q : 0;  // elements per ping-pong half
        for (int64_t u = 0; u < ((int64_t)1 << l); ++u) {
          int32_t variant = 0;
          for (int j = 0; j < l; ++j) variant |= (int32_t)(((u >> j) & 1) << S.chunk_slot[j]);
          SimJob j;
          std::memset(&j, 0, sizeof(j));
          j.state_off = l == S.c ? S.arena_off / 8 + ((uint64_t)variant << S.q)
                                 : S.tree_off / 8 + (uint64_t)(l % 2) * half + ((uint64_t)u << S.q);
          if (l > std::min(P->prefix_start, S.c)) {
            const int64_t parent = u & ((int64_t(1) << (l - 1)) - 1);
            j.src_off = S.tree_off / 8 + (uint64_t)((l - 1) % 2) * half + ((uint64_t)parent << S.q);
          } else {
            j.src_off = j.state_off;
          }
          j.pass_id = pid;
          j.variant = variant;
          j.wg_begin = L.total_wg;
          if ((int64_t)L.total_wg + nb > ((int64_t)1 << 31) - 1)
            return fail(CCUT_EUNSUPPORTED, "simulation launch exceeds 2^31 workgroups");
          L.total_wg += nb;
          P->jobs.push_back(j);
          L.n_jobs++;
        }
      }
      P->launches.push_back(L);
    }
  }
  return 0;
}

// Schedules every segment program into LDS passes of at most 2^bmax amplitudes
// and rebuilds the simulation launches and the packed table image.  The table
// region of the arena is reserved at plan creation with room for later
// rebuilds at other block sizes; a rebuild that outgrows it enlarges the arena.
int build_sim_tables(ccut_plan* P, bool first) {
  P->bmax = P->block_bits > 0 ? P->block_bits : auto_block_bits(P);
  P->prefix_on = P->prefix_mode == 1 || (P->prefix_mode < 0 && auto_prefix(P));
  P->pass_descs.clear();
  P->stage_descs.clear();
  P->kops.clear();
  P->grefs.clear();
  P->jobs.clear();
  P->launches.clear();
  for (auto& S : P->segs)
    if (int rc = schedule_passes(S.prog, P->bmax, P->low_bits, S.passes, true, P->fuse)) return rc;
  const int n_seg = P->n_seg;
  if (P->prefix_on) {
    if (int rc = build_tree_launches(P)) return rc;
  } else {
  // Simulation launches: pass p of every segment that has one, all variants.
  size_t max_passes = 0;
  for (auto& S : P->segs) max_passes = std::max(max_passes, S.passes.size());
  for (size_t p = 0; p < max_passes; ++p) {
    ccut_plan::Launch L{(int)P->jobs.size(), 0, 0};
    // largest states first so a persistent grid drains evenly
    std::vector<int> order;
    for (int i = 0; i < n_seg; ++i)
      if (P->segs[i].passes.size() > p) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return P->segs[a].q > P->segs[b].q; });
    for (int i : order) {
      auto& S = P->segs[i];
      int pid = append_pass(S.passes[p], S.q, P->pass_descs, P->stage_descs, P->kops, P->grefs, P->fuse);
      int nb = P->pass_descs[pid].n_blocks;
      for (int64_t r = 0; r < ((int64_t)1 << S.c); ++r) {
        SimJob j;
        std::memset(&j, 0, sizeof(j));
        j.state_off = S.arena_off / 8 + ((uint64_t)r << S.q);
        j.pass_id = pid;
        j.variant = (int32_t)r;
        j.wg_begin = L.total_wg;
        if ((int64_t)L.total_wg + nb > ((int64_t)1 << 31) - 1)
          return fail(CCUT_EUNSUPPORTED, "simulation launch exceeds 2^31 workgroups");
        L.total_wg += nb;
        P->jobs.push_back(j);
        L.n_jobs++;
      }
    }
    P->launches.push_back(L);
  }
  }

  for (auto& L : P->launches) {
    for (int j = L.job_begin; j < L.job_begin + L.n_jobs; ++j) {
      const PassDesc& d = P->pass_descs[P->jobs[j].pass_id];
      if (d.stage_count > 0) L.rec_cap = std::max(L.rec_cap, d.op_count + d.stage_count);
    }
  }

  pack_image(P);
  if (P->dev.blob) {  // launches already enqueued may still read the old copy: keep it until the plan is freed
    P->retired.push_back(P->dev);
    P->dev = DeviceTables();
  }
  // arena: ... | split planes | MFMA group tables | table image; both reserved with room
  // for rebuilds at other block sizes
  const uint64_t gtab_bytes = (uint64_t)P->grefs.size() * GROUP_TABLE_UINT4 * 16;
  if (first) P->gtab_reserve = align256(2 * gtab_bytes + 65536);
  P->gtab_reserve = std::max<uint64_t>(P->gtab_reserve, align256(gtab_bytes));
  // arena: states | prefix scratch | MFMA group tables | table image || merge temps | split planes
  P->gtab_off = align256(P->tree_off + P->tree_bytes);
  P->tables_off = align256(P->gtab_off + P->gtab_reserve);
  if (first) P->tables_reserve = align256(4 * (uint64_t)P->image.size() + 65536);
  P->tables_reserve = std::max<uint64_t>(P->tables_reserve, align256(P->image.size()));
  P->sim_bytes = align256(P->tables_off + P->tables_reserve);
  P->temp_off[0] = P->sim_bytes;
  P->temp_off[1] = align256(P->temp_off[0] + P->temp_bytes[0]);
  P->split_off = align256(P->temp_off[1] + P->temp_bytes[1]);
  P->total_arena = align256(P->split_off + P->split_bytes);
  return 0;
}


}  // namespace ccut

using namespace ccut;

namespace {

// Per-cut weight of Eq. (CZ): s_0 = 1/(1+i), s_1 = i/(1+i).
cd cut_weight(int bit) { return bit ? cd(0.5, 0.5) : cd(0.5, -0.5); }

void pauli_matrix(int p, cd m[4]) {
  static const cd I(0, 1);
  const cd tab[4][4] = {{1, 0, 0, 1}, {0, 1, 1, 0}, {0, -I, I, 0}, {1, 0, 0, -1}};
  for (int z = 0; z < 4; ++z) m[z] = tab[p][z];
}

// A run of boundary gates cut as one: a CZ / CX, or consecutive Pauli-rotation
// gates on the same pair (they commute, so their product is one Pauli rotation).
struct Run {
  int64_t first;
  int boundary;
  bool rotation;
  double t[3];
  cd phase;
  int n_gates;
};

// Decomposition and term weights of a cut (Eq. CZ; Eq. schmidt in the Pauli form).
ccut_plan::CutTerms cut_terms_of(const Run& r, int* n_bits) {
  ccut_plan::CutTerms ct;
  if (!r.rotation) {
    ct.form = 0;
    ct.w[0] = cut_weight(0);
    ct.w[1] = cut_weight(1);
    *n_bits = 1;
    return ct;
  }
  cd c[4];
  pauli_rotation_coeffs(r.t, c);
  for (auto& x : c) x *= r.phase;
  int nz[4], n = 0;
  for (int p = 0; p < 4; ++p)
    if (std::abs(c[p]) > 1e-12) nz[n++] = p;
  if (n <= 2) {  // Schmidt rank 2 (or 1): one bit between two Paulis
    ct.form = 1;
    ct.pa = nz[0];
    ct.pb = n == 2 ? nz[1] : (nz[0] + 1) % 4;
    ct.w[0] = c[ct.pa];
    ct.w[1] = c[ct.pb];
    *n_bits = 1;
  } else {  // rank 4: X^{b0} Z^{b1}, and Y (x) Y = -(X Z) (x) (X Z)
    ct.form = 2;
    ct.w[0] = c[0];
    ct.w[1] = c[1];
    ct.w[2] = c[3];
    ct.w[3] = -c[2];
    *n_bits = 2;
  }
  return ct;
}

}  // namespace

extern "C" int ccut_cut_plan(int32_t q, const ccut_gate_t* gates, int64_t n_gates, int32_t n_seg,
                             const int32_t* seg_sizes, ccut_plan_t** plan_out) {
  clear_error();
  if (!plan_out) return fail(CCUT_EINVAL, "plan_out is NULL");
  *plan_out = nullptr;
  if (q < 1 || q > CCUT_MAX_PLAN_Q) return fail(CCUT_EINVAL, "q=%d outside [1, %d]", q, CCUT_MAX_PLAN_Q);
  if (n_seg < 1 || n_seg > CCUT_MAX_SEG || n_seg > q)
    return fail(CCUT_EINVAL, "n_seg=%d outside [1, min(q, %d)]", n_seg, CCUT_MAX_SEG);
  if (n_gates < 0 || (n_gates > 0 && !gates)) return fail(CCUT_EINVAL, "bad gate array");
  if (n_gates > (int64_t)1 << 30) return fail(CCUT_EINVAL, "too many gates");

  ccut_plan* P = new (std::nothrow) ccut_plan();
  if (!P) return fail(CCUT_ENOMEM, "host allocation failed");
  std::unique_ptr<ccut_plan> guard(P);
  P->q = q;
  P->n_seg = n_seg;
  P->n_gates = (int32_t)n_gates;
  P->segs.resize(n_seg);
  int acc = 0;
  for (int i = 0; i < n_seg; ++i) {
    int s = seg_sizes ? seg_sizes[i] : q / n_seg + (i >= n_seg - q % n_seg ? 1 : 0);
    if (s < 1) return fail(CCUT_EINVAL, "segment %d has size %d", i, s);
    if (s > CCUT_MAX_Q) return fail(CCUT_EINVAL, "segment %d has %d qubits (max %d)", i, s, CCUT_MAX_Q);
    P->segs[i].q = s;
    P->segs[i].off = acc;
    acc += s;
  }
  if (acc != q) return fail(CCUT_EINVAL, "segment sizes add up to %d, not q=%d", acc, q);
  std::vector<int> seg_of(q);
  for (int i = 0; i < n_seg; ++i)
    for (int t = 0; t < P->segs[i].q; ++t) seg_of[P->segs[i].off + t] = i;

  // Algorithm 1: scan for boundary gates.  Pauli-rotation gates that follow each
  // other on the same cross-boundary pair, with no gate on either qubit in
  // between, join one run (one cut).
  std::vector<Run> runs;
  std::vector<int> run_of_gate(n_gates, -1);
  std::vector<uint8_t> absorbed(n_gates, 0);
  std::vector<int64_t> last_gate(q, -1);
  for (int64_t k = 0; k < n_gates; ++k) {
    const ccut_gate_t& g = gates[k];
    if (int rc = check_gate(g, q, k)) return rc;
    const bool two = is_two_qubit_kind(g.kind);
    if (two && seg_of[g.q0] != seg_of[g.q1]) {
      const int sa = seg_of[g.q0], sb = seg_of[g.q1];
      if (std::abs(sa - sb) != 1)
        return fail(CCUT_EUNCUTTABLE, "gate %lld joins non-adjacent segments %d and %d", (long long)k, sa, sb);
      const bool rot = is_pauli_rotation_kind(g.kind);
      double t[3];
      cd ph;
      if (rot) pauli_rotation_form(g, t, &ph);
      const int64_t pa = last_gate[g.q0], pb = last_gate[g.q1];
      if (rot && pa >= 0 && pa == pb && run_of_gate[pa] >= 0 && runs[run_of_gate[pa]].rotation) {
        Run& R = runs[run_of_gate[pa]];
        for (int z = 0; z < 3; ++z) R.t[z] += t[z];
        R.phase *= ph;
        R.n_gates++;
        run_of_gate[k] = run_of_gate[pa];
        absorbed[k] = 1;
      } else {
        Run R{k, std::min(sa, sb), rot, {0, 0, 0}, cd(1.0), 1};
        if (rot) {
          for (int z = 0; z < 3; ++z) R.t[z] = t[z];
          R.phase = ph;
        }
        run_of_gate[k] = (int)runs.size();
        runs.push_back(R);
      }
    }
    last_gate[g.q0] = k;
    if (two) last_gate[g.q1] = k;
  }
  std::vector<std::vector<int>> on_boundary(std::max(0, n_seg - 1));
  std::vector<ccut_plan::CutTerms> run_terms(runs.size());
  std::vector<int> run_bits(runs.size());
  for (size_t r = 0; r < runs.size(); ++r) {
    on_boundary[runs[r].boundary].push_back((int)r);
    run_terms[r] = cut_terms_of(runs[r], &run_bits[r]);
  }
  P->c_b.assign(std::max(0, n_seg - 1), 0);
  for (int b = 0; b + 1 < n_seg; ++b)
    for (int r : on_boundary[b]) P->c_b[b] += run_bits[r];
  for (int i = 0; i < n_seg; ++i) {
    auto& S = P->segs[i];
    S.c_lo = i > 0 ? P->c_b[i - 1] : 0;
    S.c_hi = i + 1 < n_seg ? P->c_b[i] : 0;
    S.c = S.c_lo + S.c_hi;
    if (S.c > CCUT_MAX_CUTS_PER_SEG)
      return fail(CCUT_EUNSUPPORTED, "segment %d has %d adjacent cut bits (max %d)", i, S.c, CCUT_MAX_CUTS_PER_SEG);
  }
  // Cut numbering: boundary-major, gate order within a boundary; each cut takes
  // n_bits consecutive variant bits.
  std::vector<int> cut_of_run(runs.size(), -1);
  P->bw.assign(std::max(0, n_seg - 1), {});
  for (int b = 0; b + 1 < n_seg; ++b) {
    int pos = 0;
    std::vector<int> cut_pos;
    for (int r : on_boundary[b]) {
      const ccut_gate_t& g = gates[runs[r].first];
      ccut_cut_info_t c;
      std::memset(&c, 0, sizeof(c));
      c.gate_index = (int32_t)runs[r].first;
      c.kind = g.kind;
      c.boundary = b;
      bool q0_low = seg_of[g.q0] == b;
      c.q_low = q0_low ? g.q0 : g.q1;
      c.q_high = q0_low ? g.q1 : g.q0;
      c.target_high = (g.kind == CCUT_GATE_CX && q0_low) ? 1 : 0;
      // segment b sees this boundary as its upper one; segment b+1 as its lower one
      c.bit_low = P->segs[b].c_lo + pos;
      c.bit_high = pos;
      c.n_bits = run_bits[r];
      c.n_gates = runs[r].n_gates;
      cut_pos.push_back(pos);
      pos += run_bits[r];
      cut_of_run[r] = (int)P->cuts.size();
      P->cuts.push_back(c);
      P->cut_terms.push_back(run_terms[r]);
    }
    // weights of the boundary's term combinations: product over its cuts
    const int64_t K = (int64_t)1 << P->c_b[b];
    P->bw[b].resize((size_t)K);
    for (int64_t m = 0; m < K; ++m) {
      cd w = 1.0;
      for (size_t j = 0; j < on_boundary[b].size(); ++j) {
        const int r = on_boundary[b][j];
        w *= run_terms[r].w[(m >> cut_pos[j]) & ((1 << run_bits[r]) - 1)];
      }
      P->bw[b][(size_t)m] = w;
    }
  }

  // Per-segment programs: the segment's own gates, plus the slot ops of each adjacent cut.
  for (int i = 0; i < n_seg; ++i) {
    auto& S = P->segs[i];
    ProgramBuilder pb(S.q);
    for (int64_t k = 0; k < n_gates; ++k) {
      const ccut_gate_t& g = gates[k];
      if (run_of_gate[k] >= 0) {
        if (absorbed[k]) continue;  // applied with the first gate of its run
        const int cj = cut_of_run[run_of_gate[k]];
        const ccut_cut_info_t& c = P->cuts[cj];
        const ccut_plan::CutTerms& ct = P->cut_terms[cj];
        int side;  // 0: this segment holds q_low, 1: q_high
        if (c.boundary == i) side = 0;
        else if (c.boundary + 1 == i) side = 1;
        else continue;
        const int local = (side == 0 ? c.q_low : c.q_high) - S.off;
        const int slot = side == 0 ? c.bit_low : c.bit_high;
        if (ct.form == 1) {
          cd m0[4], m1[4];
          pauli_matrix(ct.pa, m0);
          pauli_matrix(ct.pb, m1);
          pb.one_qubit(local, m0, m1, slot);
          continue;
        }
        if (ct.form == 2) {  // Z^{b1}, then X^{b0}
          cd id[4], x[4], z[4];
          pauli_matrix(0, id);
          pauli_matrix(1, x);
          pauli_matrix(3, z);
          pb.one_qubit(local, id, z, slot + 1);
          pb.one_qubit(local, id, x, slot);
          continue;
        }
        cd s0[4] = {1, 0, 0, cd(0, 1)}, s1[4] = {1, 0, 0, cd(0, -1)};
        bool is_target = c.kind == CCUT_GATE_CX && ((side == 1) == (c.target_high == 1));
        if (is_target) {  // H S H and H S^dag H
          const double r2 = 1.0 / std::sqrt(2.0);
          cd h[4] = {r2, r2, r2, -r2}, t0[4], t1[4];
          auto mm = [](const cd* a, const cd* b, cd* o) {
            cd r[4] = {a[0] * b[0] + a[1] * b[2], a[0] * b[1] + a[1] * b[3],
                       a[2] * b[0] + a[3] * b[2], a[2] * b[1] + a[3] * b[3]};
            for (int z = 0; z < 4; ++z) o[z] = r[z];
          };
          mm(s0, h, t0); mm(h, t0, s0);
          mm(s1, h, t1); mm(h, t1, s1);
        }
        pb.one_qubit(local, s0, s1, slot);
        continue;
      }
      if (seg_of[g.q0] != i) continue;
      pb.gate(g, S.off);
    }
    S.prog = std::move(pb.prog);
  }

  // Arena: segment-major, variant-minor, 256-byte aligned bases.
  uint64_t off = 0;
  for (auto& S : P->segs) {
    S.arena_off = off;
    off = align256(off + ((uint64_t)8 << S.q) * ((uint64_t)1 << S.c));
  }
  P->state_bytes = off;
  P->merge_ok = q <= CCUT_MAX_Q;
  P->psi_bytes = (uint64_t)8 << q;

  // Merge stages (Algorithm 3 contracted boundary by boundary).
  uint64_t ping = 0, pong = 0;
  int qacc = P->segs[0].q;
  for (int k = 0; k + 1 < n_seg; ++k) {
    const auto& Sn = P->segs[k + 1];
    MergeStage st;
    std::memset(&st, 0, sizeof(st));
    st.K = 1 << P->c_b[k];
    bool last = (k + 2 == n_seg);
    st.batch = last ? 1 : (1 << P->c_b[k + 1]);
    st.qx = qacc;
    st.qy = Sn.q;
    if (k == 0) {
      st.a_src = 0;
      st.a_off = P->segs[0].arena_off / 8;
      st.a_kstride = (uint64_t)1 << P->segs[0].q;
    } else {
      st.a_src = (k - 1) % 2 == 0 ? 1 : 2;
      st.a_off = 0;
      st.a_kstride = (uint64_t)1 << qacc;
    }
    st.a_bstride = 0;
    st.b_src = 0;
    st.b_off = Sn.arena_off / 8;
    st.b_kstride = (uint64_t)1 << Sn.q;
    st.b_bstride = (uint64_t)st.K << Sn.q;
    st.out_dst = last ? 3 : (k % 2 == 0 ? 1 : 2);
    st.out_off = 0;
    st.out_bstride = (uint64_t)1 << (qacc + Sn.q);
    st.weight_off = (int32_t)(P->weights.size() / 2);
    for (int m = 0; m < st.K; ++m) {
      const cd w = P->bw[k][(size_t)m];
      P->weights.push_back((float)w.real());
      P->weights.push_back((float)w.imag());
    }
    if (!last && P->merge_ok) {
      uint64_t bytes = ((uint64_t)8 << (qacc + Sn.q)) * (uint64_t)st.batch;
      if (k % 2 == 0) ping = std::max(ping, bytes); else pong = std::max(pong, bytes);
    }
    qacc += Sn.q;
    P->stages.push_back(st);
  }
  P->temp_bytes[0] = ping;
  P->temp_bytes[1] = pong;
  // Split-precision planes of the MFMA merge (reused stage after stage).
  P->split_bytes = 0;
  for (const MergeStage& st : P->stages) {
    if (!P->merge_ok || !merge_mfma_supported(st.qx, st.qy)) continue;
    const int S = mfma_steps(st.K);
    const uint64_t r_batch = st.a_bstride ? (uint64_t)st.batch : 1;
    const uint64_t u4 = (uint64_t)st.batch * mfma_l_plane(st.qy, S) + r_batch * mfma_r_plane(st.qx, S);
    P->split_bytes = std::max(P->split_bytes, align256(2 * 16 * u4));
  }
  // Prefix-sharing scratch: two ping-pong halves of 2^(c_i - 1) states per segment
  // (reserved in both modes, so that switching the mode keeps the arena size).
  P->tree_off = align256(P->state_bytes);
  P->tree_bytes = 0;
  for (auto& S : P->segs) {
    S.tree_off = P->tree_off + P->tree_bytes;
    if (S.c > 0) P->tree_bytes = align256(P->tree_bytes + (((uint64_t)8 << S.q) << S.c));
  }

  // MFMA merge GEMM: the column-stationary kernel up to K = 64, else the LDS-staged one
  int kmax = 1;
  for (const MergeStage& st : P->stages) kmax = std::max(kmax, st.K);
  P->merge_epilogue = kmax <= 64 ? 6 : 5;

  apply_tuned(P);
  if (int rc = build_sim_tables(P, true)) return rc;

  *plan_out = guard.release();
  return CCUT_OK;
}

extern "C" int ccut_plan_info(const ccut_plan_t* plan, ccut_plan_info_t* info) {
  clear_error();
  if (!plan || !info) return fail(CCUT_EINVAL, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->q = plan->q;
  info->n_seg = plan->n_seg;
  info->c_total = (int32_t)plan->cuts.size();
  info->n_gates = plan->n_gates;
  info->n_sub = 0;
  for (int i = 0; i < plan->n_seg; ++i) {
    const auto& S = plan->segs[i];
    info->seg_size[i] = S.q;
    info->seg_offset[i] = S.off;
    info->c_seg[i] = S.c;
    info->seg_state_offset[i] = S.arena_off;
    info->n_sub += (int64_t)1 << S.c;
  }
  for (size_t b = 0; b < plan->c_b.size(); ++b) info->c_boundary[b] = plan->c_b[b];
  int bits = 0;
  for (int c : plan->c_b) bits += c;
  info->n_terms = bits < 63 ? (int64_t)1 << bits : INT64_MAX;  // eight segments can reach 2^64
  info->state_bytes = plan->state_bytes;
  info->arena_bytes = plan->total_arena;
  info->sim_arena_bytes = plan->sim_bytes;
  info->psi_bytes = plan->psi_bytes;
  return CCUT_OK;
}

extern "C" int ccut_plan_cut(const ccut_plan_t* plan, int32_t j, ccut_cut_info_t* out) {
  clear_error();
  if (!plan || !out) return fail(CCUT_EINVAL, "NULL argument");
  if (j < 0 || j >= (int32_t)plan->cuts.size()) return fail(CCUT_EINVAL, "cut %d out of range", j);
  *out = plan->cuts[j];
  return CCUT_OK;
}

extern "C" int ccut_cut_weight(int32_t bit, double out[2]) {
  clear_error();
  if (!out || (bit != 0 && bit != 1)) return fail(CCUT_EINVAL, "bit must be 0 or 1");
  cd w = cut_weight(bit);
  out[0] = w.real();
  out[1] = w.imag();
  return CCUT_OK;
}

extern "C" int ccut_plan_cut_terms(const ccut_plan_t* plan, int32_t j, double w[8]) {
  clear_error();
  if (!plan || !w) return fail(CCUT_EINVAL, "NULL argument");
  if (j < 0 || j >= (int32_t)plan->cuts.size()) return fail(CCUT_EINVAL, "cut %d out of range", j);
  const auto& ct = plan->cut_terms[j];
  for (int t = 0; t < 4; ++t) {
    const bool used = t < (1 << plan->cuts[j].n_bits);
    w[2 * t] = used ? ct.w[t].real() : 0.0;
    w[2 * t + 1] = used ? ct.w[t].imag() : 0.0;
  }
  return CCUT_OK;
}

extern "C" void ccut_plan_free(ccut_plan_t* plan) {
  if (!plan) return;
  release_device(plan->dev);
  for (auto& t : plan->retired) release_device(t);
  if (plan->expect_host) (void)hipHostFree(plan->expect_host);
  delete plan;
}
