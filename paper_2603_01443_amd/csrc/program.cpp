// Host side: gate matrices, single-qubit fusion and LDS-pass scheduling.
//
// A segment's subcircuit (or the whole circuit, for the uncut baseline) is
// turned into a register-level program.  Consecutive single-qubit gates on a
// qubit are multiplied into one 2x2 matrix when nothing in between acts on
// the qubit non-commutingly (a diagonal gate may move back past CZs and CX
// controls, which are diagonal on that qubit).  The program is then cut into
// passes: each pass loads blocks of 2^b amplitudes spanning b qubits into LDS
// and applies every op it can without violating gate order.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "ccut_internal.h"

namespace ccut {

namespace {

void matmul2(const cd a[4], const cd b[4], cd out[4]) {  // out = a . b
  cd r[4] = {a[0] * b[0] + a[1] * b[2], a[0] * b[1] + a[1] * b[3],
             a[2] * b[0] + a[3] * b[2], a[2] * b[1] + a[3] * b[3]};
  for (int i = 0; i < 4; ++i) out[i] = r[i];
}

bool is_diag(const cd m[4]) { return m[1] == cd(0) && m[2] == cd(0); }

}  // namespace

// Qiskit conventions: Rx/Ry/Rz(t) = exp(-i t P / 2); S = diag(1, i); T = diag(1, e^{i pi/4}).
int gate_matrix(const ccut_gate_t& g, cd m[4]) {
  const double r2 = 1.0 / std::sqrt(2.0);
  const cd I(0, 1);
  switch (g.kind) {
    case CCUT_GATE_H: m[0] = r2; m[1] = r2; m[2] = r2; m[3] = -r2; return 0;
    case CCUT_GATE_X: m[0] = 0; m[1] = 1; m[2] = 1; m[3] = 0; return 0;
    case CCUT_GATE_Y: m[0] = 0; m[1] = -I; m[2] = I; m[3] = 0; return 0;
    case CCUT_GATE_Z: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -1; return 0;
    case CCUT_GATE_S: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = I; return 0;
    case CCUT_GATE_SDG: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -I; return 0;
    case CCUT_GATE_T: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = std::polar(1.0, M_PI / 4); return 0;
    case CCUT_GATE_TDG: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = std::polar(1.0, -M_PI / 4); return 0;
    case CCUT_GATE_RX: {
      double c = std::cos(g.p0 / 2), s = std::sin(g.p0 / 2);
      m[0] = c; m[1] = -I * s; m[2] = -I * s; m[3] = c; return 0;
    }
    case CCUT_GATE_RY: {
      double c = std::cos(g.p0 / 2), s = std::sin(g.p0 / 2);
      m[0] = c; m[1] = -s; m[2] = s; m[3] = c; return 0;
    }
    case CCUT_GATE_RZ:
      m[0] = std::polar(1.0, -g.p0 / 2); m[1] = 0; m[2] = 0; m[3] = std::polar(1.0, g.p0 / 2);
      return 0;
    case CCUT_GATE_RYRZ: {  // Ry(p0) . Rz(p1)
      double c = std::cos(g.p0 / 2), s = std::sin(g.p0 / 2);
      cd e0 = std::polar(1.0, -g.p1 / 2), e1 = std::polar(1.0, g.p1 / 2);
      m[0] = c * e0; m[1] = -s * e1; m[2] = s * e0; m[3] = c * e1; return 0;
    }
    default: return -1;
  }
}

bool is_two_qubit_kind(int kind) {
  return kind == CCUT_GATE_CZ || kind == CCUT_GATE_CX || is_pauli_rotation_kind(kind);
}

bool is_pauli_rotation_kind(int kind) { return kind >= CCUT_GATE_SWAP && kind <= CCUT_GATE_RZZ; }

void pauli_rotation_form(const ccut_gate_t& g, double t[3], cd* phase) {
  t[0] = t[1] = t[2] = 0.0;
  *phase = 1.0;
  switch (g.kind) {
    case CCUT_GATE_SWAP: t[0] = t[1] = t[2] = M_PI / 2; *phase = std::polar(1.0, M_PI / 4); break;
    case CCUT_GATE_ISWAP: t[0] = t[1] = -M_PI / 2; break;
    case CCUT_GATE_RXX: t[0] = g.p0; break;
    case CCUT_GATE_RYY: t[1] = g.p0; break;
    case CCUT_GATE_RZZ: t[2] = g.p0; break;
    default: break;
  }
}

void pauli_rotation_coeffs(const double t[3], cd c[4]) {
  const double cx = std::cos(t[0] / 2), sx = std::sin(t[0] / 2);
  const double cy = std::cos(t[1] / 2), sy = std::sin(t[1] / 2);
  const double cz = std::cos(t[2] / 2), sz = std::sin(t[2] / 2);
  const cd I(0, 1);
  c[0] = cx * cy * cz - I * (sx * sy * sz);
  c[1] = -I * (sx * cy * cz) + cx * sy * sz;
  c[2] = -I * (cx * sy * cz) + sx * cy * sz;
  c[3] = -I * (cx * cy * sz) + sx * sy * cz;
}

int check_gate(const ccut_gate_t& g, int q, int64_t k) {
  const bool two = is_two_qubit_kind(g.kind);
  const bool one = g.kind >= CCUT_GATE_H && g.kind <= CCUT_GATE_RYRZ;
  if (!one && !two) return fail(CCUT_EINVAL, "gate %lld: unknown kind %d", (long long)k, g.kind);
  if (g.q0 < 0 || g.q0 >= q) return fail(CCUT_EINVAL, "gate %lld: qubit %d out of range", (long long)k, g.q0);
  if (two && (g.q1 < 0 || g.q1 >= q || g.q1 == g.q0))
    return fail(CCUT_EINVAL, "gate %lld: bad second qubit %d", (long long)k, g.q1);
  return 0;
}

ProgramBuilder::ProgramBuilder(int nq)
    : last1q(nq, -1), any_since(nq, 0), nondiag_since(nq, 0) {
  prog.nq = nq;
}

void ProgramBuilder::one_qubit(int t, const cd m0[4], const cd m1[4], int slot) {
  const bool diag = is_diag(m0) && is_diag(m1);
  const int li = last1q[t];
  if (li >= 0) {
    HOp& p = prog.ops[li];
    const bool order_ok = !any_since[t] || (diag && !nondiag_since[t]);
    const bool slot_ok = slot < 0 || p.slot < 0 || p.slot == slot;
    if (order_ok && slot_ok) {
      // fused = new . previous, for each slot bit
      cd f0[4], f1[4];
      matmul2(m0, p.m[0], f0);
      matmul2(slot >= 0 ? m1 : m0, p.slot >= 0 ? p.m[1] : p.m[0], f1);
      for (int i = 0; i < 4; ++i) { p.m[0][i] = f0[i]; p.m[1][i] = f1[i]; }
      if (slot >= 0) p.slot = slot;
      p.diag = is_diag(p.m[0]) && is_diag(p.m[1]);
      return;
    }
  }
  HOp op{};
  op.kind = HOP_1Q;
  op.q0 = t;
  op.q1 = -1;
  op.slot = slot;
  for (int i = 0; i < 4; ++i) { op.m[0][i] = m0[i]; op.m[1][i] = m1[i]; }
  op.diag = diag;
  last1q[t] = (int32_t)prog.ops.size();
  any_since[t] = nondiag_since[t] = 0;
  prog.ops.push_back(op);
}

void ProgramBuilder::cz(int a, int b) {
  HOp op{};
  op.kind = HOP_CZ;
  op.q0 = a;
  op.q1 = b;
  op.diag = true;
  op.slot = -1;
  prog.ops.push_back(op);
  any_since[a] = any_since[b] = 1;
}

void ProgramBuilder::cx(int c, int t) {
  HOp op{};
  op.kind = HOP_CX;
  op.q0 = c;
  op.q1 = t;
  op.diag = false;
  op.slot = -1;
  prog.ops.push_back(op);
  any_since[c] = 1;
  any_since[t] = nondiag_since[t] = 1;
  last1q[t] = -1;  // nothing may fuse backwards past a CX target
}

void ProgramBuilder::gate(const ccut_gate_t& g, int off) {
  const int a = g.q0 - off, b = g.q1 - off;
  auto one = [&](int t, int kind, double p0) {
    ccut_gate_t h{};
    h.kind = kind;
    h.p0 = p0;
    cd m[4];
    gate_matrix(h, m);
    one_qubit(t, m, m, -1);
  };
  // exp(-i t ZZ / 2) = CX(a, b) . Rz(t) on b . CX(a, b)
  auto rzz = [&](double t) {
    cx(a, b);
    one(b, CCUT_GATE_RZ, t);
    cx(a, b);
  };
  switch (g.kind) {
    case CCUT_GATE_CZ: cz(a, b); return;
    case CCUT_GATE_CX: cx(a, b); return;
    case CCUT_GATE_SWAP: cx(a, b); cx(b, a); cx(a, b); return;
    case CCUT_GATE_RZZ: rzz(g.p0); return;
    case CCUT_GATE_RXX:  // H Z H = X
      one(a, CCUT_GATE_H, 0); one(b, CCUT_GATE_H, 0);
      rzz(g.p0);
      one(a, CCUT_GATE_H, 0); one(b, CCUT_GATE_H, 0);
      return;
    case CCUT_GATE_RYY:  // Rx(-pi/2) Z Rx(pi/2) = Y
      one(a, CCUT_GATE_RX, M_PI / 2); one(b, CCUT_GATE_RX, M_PI / 2);
      rzz(g.p0);
      one(a, CCUT_GATE_RX, -M_PI / 2); one(b, CCUT_GATE_RX, -M_PI / 2);
      return;
    case CCUT_GATE_ISWAP: {  // exp(+i pi/4 (XX + YY)) = RXX(-pi/2) RYY(-pi/2)
      ccut_gate_t h = g;
      h.kind = CCUT_GATE_RXX;
      h.p0 = -M_PI / 2;
      gate(h, off);
      h.kind = CCUT_GATE_RYY;
      gate(h, off);
      return;
    }
    default: {
      cd m[4];
      gate_matrix(g, m);
      one_qubit(a, m, m, -1);
    }
  }
}

// ----------------------------------------------------------------- passes

namespace {

// Which qubits an op needs local (acted on non-diagonally), and which it touches diagonally.
void op_roles(const HOp& op, int* nondiag, int* n_nd, int* diagq, int* n_d) {
  *n_nd = *n_d = 0;
  if (op.kind == HOP_1Q) {
    if (op.diag) diagq[(*n_d)++] = op.q0; else nondiag[(*n_nd)++] = op.q0;
  } else if (op.kind == HOP_CZ) {
    diagq[(*n_d)++] = op.q0;
    diagq[(*n_d)++] = op.q1;
  } else {  // CX: control is diagonal, target is not
    diagq[(*n_d)++] = op.q0;
    nondiag[(*n_nd)++] = op.q1;
  }
}

void put_matrix(KOp& k, const HOp& op, bool diag_form) {
  for (int s = 0; s < 2; ++s) {
    const cd* m = op.m[s];
    float* o = k.m + 8 * s;
    for (int i = 0; i < 4; ++i) { o[2 * i] = (float)m[i].real(); o[2 * i + 1] = (float)m[i].imag(); }
  }
  (void)diag_form;
}

KOp blank(int type) {
  KOp k;
  std::memset(&k, 0, sizeof(k));
  k.type = type;
  k.slot = -1;
  k.cond = -1;
  return k;
}

void set_phase_pair(KOp& k, cd p0, cd p1) {  // for both slots
  for (int s = 0; s < 2; ++s) {
    k.m[8 * s + 0] = (float)p0.real(); k.m[8 * s + 1] = (float)p0.imag();
    k.m[8 * s + 6] = (float)p1.real(); k.m[8 * s + 7] = (float)p1.imag();
  }
}

// Translate register-level ops to block-local device ops for one pass.
void localize(const Program& prog, const std::vector<int>& take, const std::vector<int32_t>& group,
              std::vector<KOp>& out) {
  std::vector<int> loc(prog.nq, -1);
  for (size_t j = 0; j < group.size(); ++j) loc[group[j]] = (int)j;
  KOp czl = blank(KOP_CZL);
  auto flush_czl = [&]() {
    if (czl.nterms > 0) out.push_back(czl);
    czl = blank(KOP_CZL);
  };
  for (int idx : take) {
    const HOp& op = prog.ops[idx];
    if (op.kind == HOP_CZ) {
      int la = loc[op.q0], lb = loc[op.q1];
      if (la >= 0 && lb >= 0) {
        int lo = std::min(la, lb), hi = std::max(la, lb);
        uint32_t shift = (uint32_t)(hi - lo);
        uint32_t* t = reinterpret_cast<uint32_t*>(czl.m);
        int found = -1;
        for (int i = 0; i < czl.nterms; ++i) if (t[2 * i] == shift) found = i;
        if (found < 0) {
          if (czl.nterms == KOP_MAX_TERMS) { flush_czl(); t = reinterpret_cast<uint32_t*>(czl.m); }
          found = czl.nterms++;
          t[2 * found] = shift;
          t[2 * found + 1] = 0;
        }
        t[2 * found + 1] ^= (1u << lo);
        continue;
      }
      flush_czl();
      if (la >= 0 || lb >= 0) {  // Z on the local qubit when the fixed one is 1
        KOp k = blank(KOP_DIAG);
        k.a = la >= 0 ? la : lb;
        k.cond = la >= 0 ? op.q1 : op.q0;
        set_phase_pair(k, 1.0, -1.0);
        out.push_back(k);
      } else {                   // both fixed: -1 on blocks where both bits are 1
        KOp k = blank(KOP_SCALAR);
        k.a = op.q0;
        k.cond = op.q1;
        set_phase_pair(k, 1.0, -1.0);
        out.push_back(k);
      }
      continue;
    }
    flush_czl();
    if (op.kind == HOP_CX) {
      int lc = loc[op.q0], lt = loc[op.q1];
      if (lc >= 0) {
        KOp k = blank(KOP_CXL);
        k.a = lc;
        k.b = lt;
        out.push_back(k);
      } else {
        KOp k = blank(KOP_DENSE);
        k.a = lt;
        k.cond = op.q0;
        k.m[2] = 1; k.m[4] = 1; k.m[10] = 1; k.m[12] = 1;  // X for both slots
        out.push_back(k);
      }
      continue;
    }
    // single-qubit
    int lt = loc[op.q0];
    KOp k = blank(op.diag ? (lt >= 0 ? KOP_DIAG : KOP_SCALAR) : KOP_DENSE);
    k.a = lt >= 0 ? lt : op.q0;
    k.slot = op.slot;
    put_matrix(k, op, op.diag);
    out.push_back(k);
  }
  flush_czl();
}

}  // namespace

// ------------------------------------------------------------ register stages

namespace {

// Local bits an op acts on non-diagonally (at most one) and diagonally.
void kop_roles(const KOp& k, int* nd, int* n_nd, int* dg, int* n_dg) {
  *n_nd = *n_dg = 0;
  switch (k.type) {
    case KOP_DENSE: nd[(*n_nd)++] = k.a; break;
    case KOP_DIAG: dg[(*n_dg)++] = k.a; break;
    case KOP_CXL: dg[(*n_dg)++] = k.a; nd[(*n_nd)++] = k.b; break;
    case KOP_CZL: {
      const uint32_t* t = reinterpret_cast<const uint32_t*>(k.m);
      uint32_t bits = 0;
      for (int i = 0; i < k.nterms; ++i) bits |= t[2 * i + 1] | (t[2 * i + 1] << t[2 * i]);
      for (int j = 0; j < 32; ++j)
        if ((bits >> j) & 1) dg[(*n_dg)++] = j;
      break;
    }
    default: break;  // KOP_SCALAR: a block-wide phase, commutes with everything
  }
}

// Adds the CZ pairs (j, j + shift) of the bits in `mask` to a KOP_CZL record.
// Returns false (record unchanged) when a new shift does not fit.
bool add_cz_terms(KOp& k, uint32_t shift, uint32_t mask) {
  if (!mask) return true;
  uint32_t* t = reinterpret_cast<uint32_t*>(k.m);
  for (int i = 0; i < k.nterms; ++i)
    if (t[2 * i] == shift) {
      t[2 * i + 1] ^= mask;  // CZ twice on one pair is the identity
      return true;
    }
  if (k.nterms == KOP_MAX_TERMS) return false;
  t[2 * k.nterms] = shift;
  t[2 * k.nterms + 1] = mask;
  ++k.nterms;
  return true;
}

// Emits one stage's items (single ops, or a KOP_GROUP with its members) in
// order, folding what acts on the register positions alone into KOP_FUSED runs:
// - a run collects groups, and diagonal phases, CZ pairs and CX gates whose bits
//   are all register bits, with at most four distinct variant slots; it becomes a
//   KOP_FUSED record (one 16x16 matrix) when it holds a group and something more;
// - diagonal ops on bits outside the register set (phases, CZ pairs with both
//   bits outside, block-wide scalars) commute with every op of the stage, whose
//   non-diagonal actions are all on register bits: they are applied after it;
// - a CZ pair with one bit inside and one outside (a Z on a register position,
//   conditioned per thread) and every other op end the run.
void emit_fused(const std::vector<std::vector<KOp>>& items, const std::vector<int>& reg,
                const std::vector<int>& pos_of, std::vector<KOp>& out) {
  const int nb = (int)pos_of.size();
  auto in_reg = [&](int j) { return j >= 0 && j < nb && pos_of[j] >= 0; };
  std::vector<KOp> run, tail;
  std::vector<int> run_slots;
  int run_groups = 0, run_other = 0;
  KOp outside = blank(KOP_CZL);
  auto flush = [&]() {
    if (run_groups >= 2 || (run_groups == 1 && run_other > 0)) {
      KOp h = blank(KOP_FUSED);
      h.a = (int32_t)run.size();
      int sl[REG_BITS] = {-1, -1, -1, -1};
      for (size_t i = 0; i < run_slots.size(); ++i) sl[i] = run_slots[i];
      h.b = sl[0];
      h.slot = sl[1];
      h.cond = sl[2];
      h.nterms = sl[3];
      int32_t bits[REG_BITS];
      for (int p = 0; p < REG_BITS; ++p) bits[p] = reg[p];
      std::memcpy(h.m, bits, sizeof(bits));
      out.push_back(h);
    }
    out.insert(out.end(), run.begin(), run.end());
    run.clear();
    run_slots.clear();
    run_groups = run_other = 0;
  };
  // slots the records would add to the run; false if more than four in all
  auto fits = [&](const std::vector<KOp>& rec, std::vector<int>& slots) {
    slots = run_slots;
    for (const KOp& k : rec)
      if (k.type != KOP_GROUP && k.slot >= 0 && std::find(slots.begin(), slots.end(), k.slot) == slots.end())
        slots.push_back(k.slot);
    return slots.size() <= (size_t)REG_BITS;
  };
  auto join = [&](const std::vector<KOp>& rec, bool group) {
    std::vector<int> slots;
    if (!fits(rec, slots) || run.size() + rec.size() > (size_t)FUSED_MAX_RECORDS) {
      flush();
      fits(rec, slots);
    }
    run_slots = slots;
    run.insert(run.end(), rec.begin(), rec.end());
    (group ? run_groups : run_other) += 1;
  };
  auto defer = [&](const KOp& k) { tail.push_back(k); };
  for (const auto& rec : items) {
    const KOp& k = rec[0];
    switch (k.type) {
      case KOP_GROUP:
        join(rec, true);
        break;
      case KOP_DIAG:
        if (!in_reg(k.a)) defer(k);
        else if (k.cond < 0) join(rec, false);
        else { flush(); out.push_back(k); }
        break;
      case KOP_SCALAR:
        defer(k);
        break;
      case KOP_CXL:
        if (in_reg(k.a)) join(rec, false);
        else { flush(); out.push_back(k); }
        break;
      case KOP_CZL: {
        KOp inside = blank(KOP_CZL), cross = blank(KOP_CZL);
        const uint32_t* t = reinterpret_cast<const uint32_t*>(k.m);
        for (int i = 0; i < k.nterms; ++i) {
          const uint32_t sh = t[2 * i], mk = t[2 * i + 1];
          uint32_t mi = 0, mc = 0, mo = 0;
          for (int j = 0; j < 32; ++j) {
            if (!((mk >> j) & 1)) continue;
            const bool a_in = in_reg(j), b_in = in_reg(j + (int)sh);
            (a_in && b_in ? mi : (a_in || b_in) ? mc : mo) |= 1u << j;
          }
          add_cz_terms(inside, sh, mi);  // at most the record's own term count
          add_cz_terms(cross, sh, mc);
          if (!add_cz_terms(outside, sh, mo)) {
            defer(outside);
            outside = blank(KOP_CZL);
            add_cz_terms(outside, sh, mo);
          }
        }
        if (inside.nterms > 0) join({inside}, false);
        if (cross.nterms > 0) {
          flush();
          out.push_back(cross);
        }
        break;
      }
      default:  // conditional 2x2 gates
        flush();
        out.push_back(k);
        break;
    }
  }
  flush();
  if (outside.nterms > 0) out.push_back(outside);
  out.insert(out.end(), tail.begin(), tail.end());
}

}  // namespace

void stage_kops(const std::vector<KOp>& kops, int b, std::vector<StageDesc>& stages, std::vector<KOp>& out,
                bool fuse) {
  std::vector<int> pending(kops.size());
  for (size_t i = 0; i < pending.size(); ++i) pending[i] = (int)i;
  while (!pending.empty()) {
    std::vector<long> need(b, (long)1 << 40);
    for (size_t pos = 0; pos < pending.size(); ++pos) {
      int nd[1], dg[32], n_nd, n_dg;
      kop_roles(kops[pending[pos]], nd, &n_nd, dg, &n_dg);
      for (int i = 0; i < n_nd; ++i) need[nd[i]] = std::min(need[nd[i]], (long)pos);
    }
    std::vector<int> cand(b);
    for (int j = 0; j < b; ++j) cand[j] = j;
    std::stable_sort(cand.begin(), cand.end(), [&](int x, int y) { return need[x] < need[y]; });
    std::vector<int> reg(cand.begin(), cand.begin() + REG_BITS);
    std::sort(reg.begin(), reg.end());
    std::vector<int> pos_of(b, -1);
    for (int k = 0; k < REG_BITS; ++k) pos_of[reg[k]] = k;
    std::vector<uint8_t> sk_any(b, 0), sk_nd(b, 0);
    std::vector<int> take, keep;
    for (int idx : pending) {
      int nd[1], dg[32], n_nd, n_dg;
      kop_roles(kops[idx], nd, &n_nd, dg, &n_dg);
      bool ok = true;
      for (int i = 0; i < n_nd; ++i) ok = ok && pos_of[nd[i]] >= 0 && !sk_any[nd[i]];
      for (int i = 0; i < n_dg; ++i) ok = ok && !sk_nd[dg[i]];
      if (ok) {
        take.push_back(idx);
      } else {
        keep.push_back(idx);
        for (int i = 0; i < n_nd; ++i) sk_any[nd[i]] = sk_nd[nd[i]] = 1;
        for (int i = 0; i < n_dg; ++i) sk_any[dg[i]] = 1;
      }
    }
    StageDesc st;
    std::memset(&st, 0, sizeof(st));
    st.op_begin = (int32_t)out.size();
    for (int k = 0; k < REG_BITS; ++k) st.reg[k] = reg[k];
    for (int e = 0; e < (1 << REG_BITS); ++e) {
      int r = 0;
      for (int k = 0; k < REG_BITS; ++k)
        if ((e >> k) & 1) r |= 1 << reg[k];
      st.roff[e] = r;
      st.proff[e] = r + (r >> 4);
    }
    // Runs of unconditional 2x2 gates on distinct register positions become one
    // KOP_GROUP (they act on different qubits, so their order inside the run is free).
    std::vector<std::vector<KOp>> items;
    for (size_t t = 0; t < take.size();) {
      const KOp& k0 = kops[take[t]];
      if (k0.type != KOP_DENSE || k0.cond >= 0) {
        KOp k = k0;
        if (k.type == KOP_DENSE) k.a = pos_of[k.a];
        if (k.type == KOP_CXL) k.b = pos_of[k.b];
        items.push_back({k});
        ++t;
        continue;
      }
      KOp members[REG_BITS];
      int mask = 0;
      while (t < take.size()) {
        const KOp& kd = kops[take[t]];
        if (kd.type != KOP_DENSE || kd.cond >= 0 || ((mask >> pos_of[kd.a]) & 1)) break;
        const int p = pos_of[kd.a];
        members[p] = kd;
        members[p].a = p;
        mask |= 1 << p;
        ++t;
      }
      KOp g = blank(KOP_GROUP);
      g.a = mask;
      for (int p = 0; p < REG_BITS; ++p) {
        if (!((mask >> p) & 1)) {  // exact identity: x * 1 + y * 0 reproduces x bit for bit
          members[p] = blank(KOP_DENSE);
          members[p].a = p;
          members[p].m[0] = members[p].m[6] = members[p].m[8] = members[p].m[14] = 1.0f;
        }
      }
      static_assert(REG_BITS == 4, "group header holds four slots");
      g.b = members[0].slot;
      g.slot = members[1].slot;
      g.cond = members[2].slot;
      g.nterms = members[3].slot;
      items.push_back({g});
      for (int p = 0; p < REG_BITS; ++p) items.back().push_back(members[p]);
    }
    const size_t first = out.size();
    if (fuse) {
      emit_fused(items, reg, pos_of, out);
    } else {
      for (const auto& rec : items) out.insert(out.end(), rec.begin(), rec.end());
    }
    for (size_t i = first; i < out.size(); ++i) {
      KOp& k = out[i];
      if (k.type != KOP_CZL) continue;
      const uint32_t* t = reinterpret_cast<const uint32_t*>(k.m);
      k.a = (int32_t)t[0];
      k.b = (int32_t)t[1];
      k.pad[0] = k.nterms > 1 ? (int32_t)t[2] : 0;
      k.pad[1] = k.nterms > 1 ? (int32_t)t[3] : 0;
    }
    st.op_count = (int32_t)out.size() - st.op_begin;
    stages.push_back(st);
    pending.swap(keep);
  }
}

int schedule_raw(const Program& prog, int bmax, int low_bits, std::vector<Pass>& out, bool from_zero);

namespace {

// Op headers plus stage heads a register-stage pass may hold: the kernel copies
// them (32 bytes each) into LDS beside its block.
int max_pass_records(int b) {
  const size_t block = sim_shmem_bytes(b, 0);
  return block >= SIM_LDS_MAX ? 0 : (int)((SIM_LDS_MAX - block) / 32);
}

// Appends p to out, split into consecutive passes over the same group until each
// one's records fit.  Later parts read the state the earlier ones wrote.
void fit_pass(Pass p, bool fuse, std::vector<Pass>& out) {
  const int b = (int)p.group.size();
  bool fits = b < STAGE_MIN_B || p.kops.size() < 2;
  if (!fits) {
    const size_t cap = (size_t)max_pass_records(b);
    fits = 6 * p.kops.size() <= cap;  // per op at most a group header, four members and a stage
    if (!fits) {
      std::vector<StageDesc> st;
      std::vector<KOp> sk;
      stage_kops(p.kops, b, st, sk, fuse);
      fits = sk.size() + st.size() <= cap;
    }
  }
  if (fits) {
    out.push_back(std::move(p));
    return;
  }
  Pass second = p;
  const size_t h = p.kops.size() / 2;
  second.kops.assign(p.kops.begin() + h, p.kops.end());
  second.init = false;
  second.from_src = false;
  p.kops.resize(h);
  fit_pass(std::move(p), fuse, out);
  fit_pass(std::move(second), fuse, out);
}

}  // namespace

int schedule_passes(const Program& prog, int bmax, int low_bits, std::vector<Pass>& out, bool from_zero,
                    bool fuse) {
  std::vector<Pass> raw;
  if (int rc = schedule_raw(prog, bmax, low_bits, raw, from_zero)) return rc;
  out.clear();
  for (Pass& p : raw) fit_pass(std::move(p), fuse, out);
  return 0;
}

int schedule_raw(const Program& prog, int bmax, int low_bits, std::vector<Pass>& out, bool from_zero) {
  out.clear();
  const int nq = prog.nq;
  std::vector<int> pending(prog.ops.size());
  for (size_t i = 0; i < pending.size(); ++i) pending[i] = (int)i;
  if (nq <= bmax) {
    Pass p;
    for (int j = 0; j < nq; ++j) p.group.push_back(j);
    p.init = from_zero;
    p.from_src = !from_zero;
    localize(prog, pending, p.group, p.kops);
    out.push_back(std::move(p));
    return 0;
  }
  const int L = std::min(low_bits, bmax);
  bool first = true;
  int guard = 0;
  while (first || !pending.empty()) {
    if (++guard > 1000000) return fail(CCUT_EINVAL, "pass scheduler made no progress");
    // qubits ordered by the position of their first pending non-diagonal use
    std::vector<long> need(nq, (long)1 << 40);
    for (size_t pos = 0; pos < pending.size(); ++pos) {
      int nd[2], dq[2], n_nd, n_d;
      op_roles(prog.ops[pending[pos]], nd, &n_nd, dq, &n_d);
      for (int i = 0; i < n_nd; ++i) need[nd[i]] = std::min(need[nd[i]], (long)pos);
    }
    std::vector<int> cand;
    for (int t = L; t < nq; ++t) cand.push_back(t);
    std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) { return need[a] < need[b]; });
    std::vector<int32_t> group;
    for (int t = 0; t < L; ++t) group.push_back(t);
    for (int i = 0; i < bmax - L; ++i) group.push_back(cand[i]);
    std::sort(group.begin() + L, group.end());
    std::vector<uint8_t> in_group(nq, 0);
    for (int t : group) in_group[t] = 1;
    std::vector<uint8_t> sk_any(nq, 0), sk_nd(nq, 0);
    std::vector<int> take, keep;
    for (int idx : pending) {
      int nd[2], dq[2], n_nd, n_d;
      op_roles(prog.ops[idx], nd, &n_nd, dq, &n_d);
      bool ok = true;
      for (int i = 0; i < n_nd; ++i) ok = ok && in_group[nd[i]] && !sk_any[nd[i]];
      for (int i = 0; i < n_d; ++i) ok = ok && !sk_nd[dq[i]];
      if (ok) {
        take.push_back(idx);
      } else {
        keep.push_back(idx);
        for (int i = 0; i < n_nd; ++i) sk_any[nd[i]] = sk_nd[nd[i]] = 1;
        for (int i = 0; i < n_d; ++i) sk_any[dq[i]] = 1;
      }
    }
    if (take.empty() && !first) return fail(CCUT_EINVAL, "pass scheduler made no progress");
    Pass p;
    p.group = group;
    p.init = first && from_zero;
    p.from_src = first && !from_zero;
    localize(prog, take, group, p.kops);
    out.push_back(std::move(p));
    pending.swap(keep);
    first = false;
  }
  return 0;
}

}  // namespace ccut
