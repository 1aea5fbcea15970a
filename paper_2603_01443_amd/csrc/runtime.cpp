// Runtime around the kernels: HIP-graph capture of a plan's whole pipeline,
// launch configuration, and a measuring autotuner with a persistent cache.
#include <algorithm>
#include <cmath>
#include <array>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <new>
#include <mutex>
#include <string>
#include <vector>

#include "plan.h"

struct ccut_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = -1;
  ccut::DeviceTables tables;  // the graph's own copy of the tables its kernels read
  uint64_t layout = 0;        // launch layout of the captured plan (ccut::layout_key)
};

namespace ccut {

namespace {

struct TuneEntry {
  int threads = 1024;
  int grid_cap = 0;
  int mfma_min_k = -1;
  int mfma_mode = CCUT_PREC_FP16X3;
  int epilogue = 0;
  int merge_grid = 0;
  int block_bits = 0;
  int prefix = -1;
};

std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;

// arithmetics CCUT_PREC_AUTO may take on MFMA: the two fully split ones, or FP16X2 by opt-in
bool auto_mode_ok(int m) { return m == CCUT_PREC_FP16X3 || m == CCUT_PREC_BF16X3 || m == CCUT_PREC_FP16X2; }

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  return a.substr(0, a.find(':'));
}

// Shape signature of a plan: segment sizes, variants, fused program lengths and
// merge stages (nothing that depends on the launch configuration).
std::string signature(const ccut_plan* P) {
  std::string s = "q" + std::to_string(P->q);
  for (const auto& S : P->segs)
    s += "|" + std::to_string(S.q) + "x" + std::to_string(1 << S.c) + "g" + std::to_string(S.prog.ops.size());
  for (const auto& st : P->stages)
    s += "|m" + std::to_string(st.qx) + "," + std::to_string(st.qy) + "," + std::to_string(st.K) + "," +
         std::to_string(st.batch);
  return s;
}

// Median device time of `reps` calls of fn (after one warm-up call).  `pre`, when
// given, runs untimed before every call of fn, so that fn is timed in the state the
// pipeline leaves it in (a merge right after the simulation that feeds it).
int time_call(hipStream_t s, int reps, float* ms_out, const std::function<int()>& fn,
              const std::function<int()>& pre = nullptr) {
  hipEvent_t a, b;
  CCUT_HIP(hipEventCreate(&a));
  CCUT_HIP(hipEventCreate(&b));
  int rc = pre ? pre() : 0;
  if (rc == 0) rc = fn();  // warm-up
  std::vector<float> t;
  for (int r = 0; r < reps && rc == 0; ++r) {
    if (pre && (rc = pre()) != 0) break;
    (void)hipEventRecord(a, s);
    rc = fn();
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    t.push_back(ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc) return rc;
  std::sort(t.begin(), t.end());
  *ms_out = t[t.size() / 2];
  return 0;
}

uint64_t mix(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

// Everything a captured pipeline bakes into its launches besides the contents of
// the tables: plan shape, launch configuration, arena layout, table image layout.
// Two plans with equal keys run the same launches on tables of the same layout.
uint64_t layout_key(const ccut_plan* P) {
  uint64_t h = 1469598103934665603ull;
  const std::string sig = signature(P);
  h = mix(h, sig.data(), sig.size());
  const uint64_t u[] = {P->image.size(), P->img_ops,    P->img_passes,  P->img_stages, P->img_jobs,
                        P->img_weights,  P->img_grefs,  P->tables_off,  P->gtab_off,   P->tree_off,
                        P->split_off,    P->temp_off[0], P->temp_off[1], P->total_arena, P->psi_bytes};
  h = mix(h, u, sizeof(u));
  const int32_t v[] = {P->bmax, P->prefix_on ? 1 : 0, P->prefix_start, P->sim_threads, P->sim_grid_cap,
                       P->sim_per_variant, P->sim_precision, P->merge_epilogue, P->merge_grid_cap,
                       P->auto_mfma_min_k, P->auto_mfma_mode, (int32_t)P->grefs.size(), P->fuse ? 1 : 0};
  h = mix(h, v, sizeof(v));
  for (const auto& L : P->launches) h = mix(h, &L, sizeof(L));
  for (const auto& st : P->stages) h = mix(h, &st, sizeof(st));
  for (const auto& S : P->segs) {
    const uint64_t o[2] = {S.arena_off, S.tree_off};
    h = mix(h, o, sizeof(o));
  }
  return h;
}

}  // namespace

// Applies a cached configuration to a freshly built plan, if one exists.
void apply_tuned(ccut_plan* P) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tune.empty()) return;
  auto it = g_tune.find(arch_name() + "|" + signature(P));
  if (it == g_tune.end()) return;
  P->sim_threads = it->second.threads;
  P->sim_grid_cap = it->second.grid_cap;
  P->auto_mfma_min_k = it->second.mfma_min_k;
  P->auto_mfma_mode = it->second.mfma_mode;
  P->merge_epilogue = it->second.epilogue;
  P->merge_grid_cap = it->second.merge_grid;
  P->block_bits = it->second.block_bits;
  // prefix: -1 automatic, 0 off, 1 + L on with the tree starting at level L
  P->prefix_mode = it->second.prefix <= 0 ? it->second.prefix : 1;
  P->prefix_start = it->second.prefix > 0 ? it->second.prefix - 1 : 0;
}

}  // namespace ccut

using namespace ccut;

extern "C" int ccut_plan_set_launch(ccut_plan_t* plan, int32_t threads, int32_t grid_cap, int32_t per_variant,
                                    int32_t mfma_min_terms) {
  clear_error();
  if (!plan) return fail(CCUT_EINVAL, "plan is NULL");
  if (threads != 256 && threads != 512 && threads != 1024) return fail(CCUT_EINVAL, "threads must be 256/512/1024");
  if (grid_cap < 0 || mfma_min_terms < -1) return fail(CCUT_EINVAL, "bad launch configuration");
  plan->sim_threads = threads;
  plan->sim_grid_cap = grid_cap;
  plan->sim_per_variant = per_variant ? 1 : 0;
  plan->auto_mfma_min_k = mfma_min_terms;
  return CCUT_OK;
}

extern "C" int ccut_plan_set_merge(ccut_plan_t* plan, int32_t epilogue, int32_t grid_cap) {
  clear_error();
  if (!plan) return fail(CCUT_EINVAL, "plan is NULL");
  if (epilogue < 0 || epilogue > MERGE_VARIANTS - 1 || grid_cap < 0) return fail(CCUT_EINVAL, "bad merge configuration");
  plan->merge_epilogue = epilogue;
  plan->merge_grid_cap = grid_cap;
  return CCUT_OK;
}

extern "C" int ccut_plan_work(const ccut_plan_t* plan, double out[5]) {
  clear_error();
  if (!plan || !out) return fail(CCUT_EINVAL, "NULL argument");
  for (int i = 0; i < 5; ++i) out[i] = 0.0;
  // per pass descriptor: (dense 2x2, diagonal, permutation / sign) op counts
  std::vector<std::array<int64_t, 3>> per(plan->pass_descs.size(), std::array<int64_t, 3>{0, 0, 0});
  for (size_t d = 0; d < plan->pass_descs.size(); ++d) {
    const PassDesc& pd = plan->pass_descs[d];
    for (int i = pd.op_begin; i < pd.op_begin + pd.op_count; ++i) {
      const KOp& k = plan->kops[i];
      if (k.type == KOP_FUSED) continue;  // header only: its records follow
      if (k.type == KOP_GROUP) {
        per[d][0] += __builtin_popcount((unsigned)k.a);
        i += REG_BITS;  // its member records
      } else if (k.type == KOP_DENSE) {
        ++per[d][0];
      } else if (k.type == KOP_DIAG || k.type == KOP_SCALAR) {
        ++per[d][1];
      } else {
        ++per[d][2];
      }
    }
  }
  for (const SimJob& j : plan->jobs) {
    const PassDesc& pd = plan->pass_descs[j.pass_id];
    const double amps = std::ldexp(1.0, pd.nq);
    for (int t = 0; t < 3; ++t) out[t] += (double)per[j.pass_id][t] * amps;
    out[3] += amps * (pd.init ? 1.0 : 2.0);
  }
  for (const auto& S : plan->segs) {
    int64_t dense = 0;
    for (const HOp& h : S.prog.ops) dense += h.kind == HOP_1Q && !h.diag;
    out[4] += (double)dense * std::ldexp(1.0, S.q + S.c);
  }
  return CCUT_OK;
}

extern "C" int ccut_plan_set_auto_precision(ccut_plan_t* plan, int32_t precision) {
  clear_error();
  if (!plan) return fail(CCUT_EINVAL, "plan is NULL");
  if (!auto_mode_ok(precision))
    return fail(CCUT_EINVAL, "AUTO merges on MFMA in FP16X3, BF16X3 or FP16X2, not %d", precision);
  plan->auto_mfma_mode = precision;
  return CCUT_OK;
}

extern "C" int ccut_plan_get_auto_precision(const ccut_plan_t* plan, int32_t* out) {
  clear_error();
  if (!plan || !out) return fail(CCUT_EINVAL, "NULL argument");
  *out = plan->auto_mfma_mode;
  return CCUT_OK;
}

extern "C" int ccut_plan_stats(const ccut_plan_t* plan, int64_t out[8]) {
  clear_error();
  if (!plan || !out) return fail(CCUT_EINVAL, "NULL argument");
  int64_t dense = 0, diag = 0;
  for (size_t i = 0; i < plan->kops.size(); ++i) {
    const KOp& k = plan->kops[i];
    if (k.type == KOP_FUSED) continue;  // header only: its records follow
    if (k.type == KOP_GROUP) {
      dense += __builtin_popcount((unsigned)k.a);
      i += REG_BITS;  // its member records
    } else if (k.type == KOP_DENSE || k.type == KOP_CXL) {
      ++dense;
    } else {
      ++diag;
    }
  }
  int64_t hops = 0;
  for (const auto& S : plan->segs) hops += (int64_t)S.prog.ops.size();
  out[0] = (int64_t)plan->pass_descs.size();
  out[1] = (int64_t)plan->stage_descs.size();
  out[2] = (int64_t)plan->kops.size();
  out[3] = dense;
  out[4] = diag;
  out[5] = hops;
  out[6] = (int64_t)plan->launches.size();
  out[7] = (int64_t)plan->jobs.size();
  return CCUT_OK;
}

extern "C" int ccut_plan_set_block_bits(ccut_plan_t* plan, int32_t bits) {
  clear_error();
  if (!plan) return fail(CCUT_EINVAL, "plan is NULL");
  if (bits != 0 && (bits <= plan->low_bits || bits > PASS_MAX_B))
    return fail(CCUT_EINVAL, "block bits %d outside (%d, %d] (0: automatic)", bits, plan->low_bits, PASS_MAX_B);
  const int saved = plan->block_bits;
  plan->block_bits = bits;
  if (int rc = build_sim_tables(plan, false)) {
    plan->block_bits = saved;
    (void)build_sim_tables(plan, false);
    return rc;
  }
  return CCUT_OK;
}

extern "C" int ccut_plan_set_sim_precision(ccut_plan_t* plan, int32_t precision) {
  clear_error();
  if (!plan) return fail(CCUT_EINVAL, "plan is NULL");
  if (precision != CCUT_SIM_FP32 && precision != CCUT_SIM_FP16X3)
    return fail(CCUT_EINVAL, "unknown simulation precision %d", precision);
  plan->sim_precision = precision;
  return CCUT_OK;
}

extern "C" int ccut_plan_get_sim_precision(const ccut_plan_t* plan, int32_t* out) {
  clear_error();
  if (!plan || !out) return fail(CCUT_EINVAL, "NULL argument");
  *out = plan->sim_precision;
  return CCUT_OK;
}

extern "C" int ccut_plan_set_prefix_sharing(ccut_plan_t* plan, int32_t mode) {
  clear_error();
  if (!plan) return fail(CCUT_EINVAL, "plan is NULL");
  if (mode < -1 || mode > 1) return fail(CCUT_EINVAL, "prefix sharing mode %d (0 off, 1 on, -1 automatic)", mode);
  const int saved = plan->prefix_mode;
  plan->prefix_mode = mode;
  if (int rc = build_sim_tables(plan, false)) {
    plan->prefix_mode = saved;
    (void)build_sim_tables(plan, false);
    return rc;
  }
  return CCUT_OK;
}

extern "C" int ccut_plan_set_prefix_start(ccut_plan_t* plan, int32_t level) {
  clear_error();
  if (!plan) return fail(CCUT_EINVAL, "plan is NULL");
  if (level < 0 || level > CCUT_MAX_CUTS_PER_SEG)
    return fail(CCUT_EINVAL, "prefix start level %d outside [0, %d]", level, CCUT_MAX_CUTS_PER_SEG);
  const int saved = plan->prefix_start;
  plan->prefix_start = level;
  if (int rc = build_sim_tables(plan, false)) {
    plan->prefix_start = saved;
    (void)build_sim_tables(plan, false);
    return rc;
  }
  return CCUT_OK;
}

extern "C" int ccut_plan_get_prefix_start(const ccut_plan_t* plan, int32_t* out) {
  clear_error();
  if (!plan || !out) return fail(CCUT_EINVAL, "NULL argument");
  *out = plan->prefix_start;
  return CCUT_OK;
}

extern "C" int ccut_plan_set_fusion(ccut_plan_t* plan, int32_t on) {
  clear_error();
  if (!plan) return fail(CCUT_EINVAL, "plan is NULL");
  if (on != 0 && on != 1) return fail(CCUT_EINVAL, "fusion %d (0 off, 1 on)", on);
  const bool saved = plan->fuse;
  plan->fuse = on == 1;
  if (int rc = build_sim_tables(plan, false)) {
    plan->fuse = saved;
    (void)build_sim_tables(plan, false);
    return rc;
  }
  return CCUT_OK;
}

extern "C" int ccut_plan_get_fusion(const ccut_plan_t* plan, int32_t* out) {
  clear_error();
  if (!plan || !out) return fail(CCUT_EINVAL, "NULL argument");
  *out = plan->fuse ? 1 : 0;
  return CCUT_OK;
}

extern "C" int ccut_plan_get_prefix_sharing(const ccut_plan_t* plan, int32_t* out) {
  clear_error();
  if (!plan || !out) return fail(CCUT_EINVAL, "NULL argument");
  *out = plan->prefix_on ? 1 : 0;
  return CCUT_OK;
}

extern "C" int ccut_plan_get_block_bits(const ccut_plan_t* plan, int32_t* out) {
  clear_error();
  if (!plan || !out) return fail(CCUT_EINVAL, "NULL argument");
  *out = plan->bmax;
  return CCUT_OK;
}

extern "C" int ccut_plan_get_merge(const ccut_plan_t* plan, int32_t out[2]) {
  clear_error();
  if (!plan || !out) return fail(CCUT_EINVAL, "NULL argument");
  out[0] = plan->merge_epilogue;
  out[1] = plan->merge_grid_cap;
  return CCUT_OK;
}

extern "C" int ccut_plan_get_launch(const ccut_plan_t* plan, int32_t out[4]) {
  clear_error();
  if (!plan || !out) return fail(CCUT_EINVAL, "NULL argument");
  out[0] = plan->sim_threads;
  out[1] = plan->sim_grid_cap;
  out[2] = plan->sim_per_variant;
  out[3] = plan->auto_mfma_min_k;
  return CCUT_OK;
}

extern "C" int ccut_autotune(ccut_plan_t* plan, void* d_arena, uint64_t arena_bytes, void* d_psi,
                             uint64_t psi_bytes, int32_t reps, void* stream, double* best_ms) {
  clear_error();
  if (!plan || !d_arena || !d_psi || reps < 1) return fail(CCUT_EINVAL, "bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int saved_pv = plan->sim_per_variant;
  plan->sim_per_variant = 0;
  float best = 1e30f;
  int bt = plan->sim_threads, bg = plan->sim_grid_cap, bb = plan->bmax, bpre = plan->prefix_on ? 1 : 0;
  int bstart = plan->prefix_start;
  const int saved_bits = plan->block_bits, saved_prefix = plan->prefix_mode, saved_start = plan->prefix_start;
  bool any_cut = false;
  for (const auto& S : plan->segs) any_cut = any_cut || S.c > 0;
  const int threads[3] = {256, 512, 1024};
  const int caps[5] = {0, 256, 512, 1024, 2048};
  int qmax = 0;
  for (const auto& S : plan->segs) qmax = std::max(qmax, S.q);
  // prefix sharing off / on (tree from level 0, 2, 3 or 4) x block sizes: whole segment
  // states in LDS, then 2 and 4 blocks
  int cmax = 0;
  for (const auto& S : plan->segs) cmax = std::max(cmax, S.c);
  // tree starts: the full tree, a few early levels, and the last two levels (only the
  // final slots shared)
  std::vector<std::array<int, 2>> pre_modes = {{0, 0}};
  if (any_cut)
    for (int st : {0, 2, 3, 4, cmax - 2, cmax - 1})
      if (st >= 0 && (st == 0 || st < cmax) &&
          std::find(pre_modes.begin(), pre_modes.end(), std::array<int, 2>{1, st}) == pre_modes.end())
        pre_modes.push_back({1, st});
  for (size_t pm = 0; pm < pre_modes.size(); ++pm)
  for (int bits = std::min(qmax, PASS_MAX_B); bits >= std::max(plan->low_bits + 1, std::min(qmax, PASS_MAX_B) - 2);
       --bits) {
    const int pre = pre_modes[pm][0], start = pre_modes[pm][1];
    plan->block_bits = bits;
    plan->prefix_mode = pre;
    plan->prefix_start = start;
    if (int rc = build_sim_tables(plan, false)) {
      plan->sim_per_variant = saved_pv;
      plan->block_bits = saved_bits;
      plan->prefix_mode = saved_prefix;
      plan->prefix_start = saved_start;
      (void)build_sim_tables(plan, false);
      return rc;
    }
    if (plan->total_arena > arena_bytes) continue;  // tables do not fit this caller's arena
    int total_wg = 0;
    for (const auto& L : plan->launches) total_wg = std::max(total_wg, L.total_wg);
    for (int t : threads) {
      for (int c : caps) {
        if (c != 0 && c >= total_wg) continue;
        plan->sim_threads = t;
        plan->sim_grid_cap = c;
        float ms = 0.f;
        int rc = time_call(s, reps, &ms, [&]() { return ccut_simulate_subcircuits(plan, d_arena, arena_bytes, stream); });
        if (rc == CCUT_EUNSUPPORTED) continue;  // a configuration the launch refuses: not a candidate
        if (rc) {
          plan->sim_per_variant = saved_pv;
          plan->block_bits = saved_bits;
          plan->prefix_mode = saved_prefix;
          plan->prefix_start = saved_start;
          (void)build_sim_tables(plan, false);
          return rc;
        }
        if (ms < best) { best = ms; bt = t; bg = c; bb = bits; bpre = pre; bstart = start; }
      }
    }
  }
  plan->sim_threads = bt;
  plan->sim_grid_cap = bg;
  plan->block_bits = bb;
  plan->prefix_mode = bpre;
  plan->prefix_start = bpre ? bstart : 0;
  if (int rc = build_sim_tables(plan, false)) {
    plan->sim_per_variant = saved_pv;
    return rc;
  }
  // merge: float32 vector kernel against the fully split MFMA GEMM (the CCUT_PREC_AUTO
  // arithmetic: fp16 or bf16 halves, hi.hi + hi.lo + lo.hi) at this plan's term counts,
  // over both split arithmetics, the GEMM variants and grids
  float t32 = 0.f, tmf = 1e30f;
  // every merge is timed right after a simulation, as the pipeline runs it: back to back
  // merges see the previous merge's writes still draining and rank the variants differently
  auto sim = [&]() { return ccut_simulate_subcircuits(plan, d_arena, arena_bytes, stream); };
  int rc = time_call(
      s, reps, &t32,
      [&]() { return ccut_merge_full_state(plan, d_arena, arena_bytes, d_psi, psi_bytes, CCUT_PREC_FP32, stream); },
      sim);
  int best_epi = plan->merge_epilogue, best_grid = plan->merge_grid_cap, best_mode = plan->auto_mfma_mode;
  const int saved_epi = best_epi, saved_grid = best_grid, saved_mode = best_mode;
  // Merges are short and their clocks drift while the device heats up: every candidate
  // is timed in a forward and a backward sweep (median of at least 7 runs each) and
  // keeps the better of its two medians.
  std::vector<std::array<int, 3>> cands;  // (arithmetic, variant, grid)
  for (int mode : {CCUT_PREC_FP16X3, CCUT_PREC_BF16X3})
    for (int epi = 0; epi < MERGE_VARIANTS; ++epi)
      for (int gc : {0, 512, 1024, 2048})
        if (epi < 4 || gc == 0) cands.push_back({mode, epi, gc});  // variants 4 and 5 size their own grid
  std::vector<float> tbest(cands.size(), 1e30f);
  const int mreps = std::max(reps, 7);
  for (int sweep = 0; sweep < 2 && !rc; ++sweep) {
    for (size_t j = 0; j < cands.size() && !rc; ++j) {
      const size_t i = sweep == 0 ? j : cands.size() - 1 - j;
      plan->merge_epilogue = cands[i][1];
      plan->merge_grid_cap = cands[i][2];
      const int mode = cands[i][0];
      float t = 0.f;
      rc = time_call(
          s, mreps, &t,
          [&]() { return ccut_merge_full_state(plan, d_arena, arena_bytes, d_psi, psi_bytes, mode, stream); }, sim);
      if (!rc) tbest[i] = std::min(tbest[i], t);
    }
  }
  // fp16x3 keeps ~22 significant bits against bf16x3's ~16 (both far inside 1 - F <= 1e-6 at the
  // measured shapes): bf16x3 must be more than 2 % faster
  auto weight = [&](size_t i) { return tbest[i] * (cands[i][0] == CCUT_PREC_BF16X3 ? 1.02f : 1.0f); };
  float wbest = 1e30f;
  for (size_t i = 0; i < cands.size() && !rc; ++i)
    if (weight(i) < wbest) {
      wbest = weight(i);
      tmf = tbest[i];
      best_mode = cands[i][0];
      best_epi = cands[i][1];
      best_grid = cands[i][2];
    }
  // the plan's own choice stays unless another is clearly faster: near ties would
  // otherwise flip with run-to-run noise
  for (size_t i = 0; i < cands.size() && !rc; ++i)
    if (cands[i][0] == saved_mode && cands[i][1] == saved_epi && cands[i][2] == saved_grid &&
        weight(i) <= 1.02f * wbest) {
      tmf = tbest[i];
      best_mode = saved_mode;
      best_epi = saved_epi;
      best_grid = saved_grid;
    }
  plan->merge_epilogue = best_epi;
  plan->merge_grid_cap = best_grid;
  plan->auto_mfma_mode = best_mode;
  plan->sim_per_variant = saved_pv;
  if (rc) return rc;
  int kmax = 1;
  for (const auto& st : plan->stages) kmax = std::max(kmax, st.K);
  plan->auto_mfma_min_k = tmf < t32 ? 1 : kmax + 1;
  if (best_ms) *best_ms = best + std::min(t32, tmf);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[arch_name() + "|" + signature(plan)] =
      TuneEntry{bt, bg, plan->auto_mfma_min_k, best_mode, best_epi, best_grid, bb, bpre ? 1 + plan->prefix_start : 0};
  return CCUT_OK;
}

extern "C" int ccut_autotune_save(const char* path) {
  clear_error();
  if (!path) return fail(CCUT_EINVAL, "path is NULL");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(CCUT_EINVAL, "cannot write %s", path);
  std::fprintf(f, "# ccut autotune cache: key threads grid_cap mfma_min_k epilogue merge_grid block_bits prefix "
                 "mfma_mode\n");
  for (const auto& kv : g_tune)
    std::fprintf(f, "%s %d %d %d %d %d %d %d %d\n", kv.first.c_str(), kv.second.threads, kv.second.grid_cap,
                 kv.second.mfma_min_k, kv.second.epilogue, kv.second.merge_grid, kv.second.block_bits,
                 kv.second.prefix, kv.second.mfma_mode);
  std::fclose(f);
  return CCUT_OK;
}

extern "C" int ccut_autotune_load(const char* path) {
  clear_error();
  if (!path) return fail(CCUT_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(CCUT_EINVAL, "cannot read %s", path);
  char key[1024];
  int t, c, k, ep, mg, bb, pf, mm;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  char line[1200];
  while (std::fgets(line, sizeof(line), f)) {
    if (line[0] == '#') continue;
    // the last field (AUTO's split arithmetic) is absent in caches written before it existed
    mm = CCUT_PREC_FP16X3;
    const int nf = std::sscanf(line, "%1023s %d %d %d %d %d %d %d %d", key, &t, &c, &k, &ep, &mg, &bb, &pf, &mm);
    if ((nf == 8 || nf == 9) && (t == 256 || t == 512 || t == 1024) && c >= 0 && k >= -1 && ep >= 0 &&
        ep < MERGE_VARIANTS && mg >= 0 && (bb == 0 || (bb > 4 && bb <= PASS_MAX_B)) && pf >= -1 &&
        pf <= 1 + CCUT_MAX_CUTS_PER_SEG && auto_mode_ok(mm))
      g_tune[key] = TuneEntry{t, c, k, mm, ep, mg, bb, pf};
  }
  std::fclose(f);
  return CCUT_OK;
}

extern "C" int ccut_graph_create(ccut_plan_t* plan, void* d_arena, uint64_t arena_bytes, void* d_psi,
                                 uint64_t psi_bytes, int32_t precision, void* stream, ccut_graph_t** out) {
  clear_error();
  if (!plan || !d_arena || !d_psi || !out) return fail(CCUT_EINVAL, "NULL argument");
  if (!stream) return fail(CCUT_EINVAL, "graph capture needs a non-default stream");
  *out = nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::unique_ptr<ccut_graph> G(new (std::nothrow) ccut_graph());
  if (!G) return fail(CCUT_ENOMEM, "host allocation failed");
  CCUT_HIP(hipGetDevice(&G->device));
  // the graph's kernels read its own table copy (copied now: nothing is copied from the
  // host inside the graph; ccut_graph_rebind refills it for another plan of this layout)
  if (int rc = upload_tables(G->tables, plan->image, plan->img_ops, plan->img_passes, plan->img_stages,
                             plan->img_jobs, plan->img_weights, plan->img_grefs))
    return rc;
  auto drop = [&]() {
    if (G->graph) (void)hipGraphDestroy(G->graph);
    G->graph = nullptr;
    release_device(G->tables);
  };
  // capture against the graph's copy: the plan's device tables are swapped for the capture
  const DeviceTables saved = plan->dev;
  plan->dev = G->tables;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    plan->dev = saved;
    drop();
    return hip_fail(e, "hipStreamBeginCapture");
  }
  int rc = ccut_simulate_subcircuits(plan, d_arena, arena_bytes, stream);
  if (rc == 0) rc = ccut_merge_full_state(plan, d_arena, arena_bytes, d_psi, psi_bytes, precision, stream);
  std::string msg = rc ? ccut_last_error() : "";
  e = hipStreamEndCapture(s, &G->graph);
  plan->dev = saved;
  if (rc || e != hipSuccess) {
    drop();
    return rc ? fail(rc, "%s", msg.c_str()) : hip_fail(e, "hipStreamEndCapture");
  }
  e = hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop();
    return hip_fail(e, "hipGraphInstantiate");
  }
  G->layout = layout_key(plan);
  *out = G.release();
  return CCUT_OK;
}

extern "C" int ccut_graph_rebind(ccut_graph_t* g, const ccut_plan_t* plan, void* stream) {
  clear_error();
  if (!g || !g->exec || !plan) return fail(CCUT_EINVAL, "NULL argument");
  int dev = 0;
  CCUT_HIP(hipGetDevice(&dev));
  if (dev != g->device) return fail(CCUT_EINVAL, "the graph was captured on device %d, not %d", g->device, dev);
  if (layout_key(plan) != g->layout)
    return fail(CCUT_EINVAL, "the plan's launch layout (shape, launch configuration, table layout) differs "
                "from the captured plan's");
  return staged_copy(g->tables.blob, plan->image.data(), plan->image.size(), static_cast<hipStream_t>(stream));
}

extern "C" int ccut_graph_launch(ccut_graph_t* g, void* stream) {
  clear_error();
  if (!g || !g->exec) return fail(CCUT_EINVAL, "graph is NULL");
  CCUT_HIP(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
  return CCUT_OK;
}

extern "C" void ccut_graph_free(ccut_graph_t* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  release_device(g->tables);
  delete g;
}
