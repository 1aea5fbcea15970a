// Runtime around the kernels: HIP-graph capture of a plan's whole pipeline,
// launch configuration, and a measuring autotuner with a persistent cache.
#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <new>
#include <mutex>
#include <string>
#include <vector>

#include "plan.h"

struct ccut_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = -1;
};

namespace ccut {

namespace {

struct TuneEntry {
  int threads = 1024;
  int grid_cap = 0;
  int mfma_min_k = -1;
  int epilogue = 0;
  int merge_grid = 0;
  int block_bits = 0;
  int prefix = -1;
};

std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;

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

extern "C" int ccut_plan_stats(const ccut_plan_t* plan, int64_t out[8]) {
  clear_error();
  if (!plan || !out) return fail(CCUT_EINVAL, "NULL argument");
  int64_t dense = 0, diag = 0;
  for (size_t i = 0; i < plan->kops.size(); ++i) {
    const KOp& k = plan->kops[i];
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
  // merge: float32 vector kernel against the split MFMA kernel (the CCUT_PREC_AUTO mode) at this
  // plan's term counts, over the GEMM variants and grids
  float t32 = 0.f, tmf = 1e30f;
  // every merge is timed right after a simulation, as the pipeline runs it: back to back
  // merges see the previous merge's writes still draining and rank the variants differently
  auto sim = [&]() { return ccut_simulate_subcircuits(plan, d_arena, arena_bytes, stream); };
  int rc = time_call(
      s, reps, &t32,
      [&]() { return ccut_merge_full_state(plan, d_arena, arena_bytes, d_psi, psi_bytes, CCUT_PREC_FP32, stream); },
      sim);
  int best_epi = plan->merge_epilogue, best_grid = plan->merge_grid_cap;
  const int saved_epi = best_epi, saved_grid = best_grid;
  // Merges are short and their clocks drift while the device heats up: every candidate
  // is timed in a forward and a backward sweep (median of at least 7 runs each) and
  // keeps the better of its two medians.
  std::vector<std::array<int, 2>> cands;
  for (int epi = 0; epi < 4; ++epi)
    for (int gc : {0, 512, 1024, 2048}) cands.push_back({epi, gc});
  std::vector<float> tbest(cands.size(), 1e30f);
  const int mreps = std::max(reps, 7);
  for (int sweep = 0; sweep < 2 && !rc; ++sweep) {
    for (size_t j = 0; j < cands.size() && !rc; ++j) {
      const size_t i = sweep == 0 ? j : cands.size() - 1 - j;
      plan->merge_epilogue = cands[i][0];
      plan->merge_grid_cap = cands[i][1];
      float t = 0.f;
      rc = time_call(
          s, mreps, &t,
          [&]() {
            return ccut_merge_full_state(plan, d_arena, arena_bytes, d_psi, psi_bytes, CCUT_PREC_FP16X2, stream);
          },
          sim);
      if (!rc) tbest[i] = std::min(tbest[i], t);
    }
  }
  for (size_t i = 0; i < cands.size() && !rc; ++i)
    if (tbest[i] < tmf) { tmf = tbest[i]; best_epi = cands[i][0]; best_grid = cands[i][1]; }
  // the plan's own choice stays unless another is clearly faster: near ties would
  // otherwise flip with run-to-run noise
  for (size_t i = 0; i < cands.size() && !rc; ++i)
    if (cands[i][0] == saved_epi && cands[i][1] == saved_grid && tbest[i] <= 1.02f * tmf) {
      tmf = tbest[i];
      best_epi = saved_epi;
      best_grid = saved_grid;
    }
  plan->merge_epilogue = best_epi;
  plan->merge_grid_cap = best_grid;
  plan->sim_per_variant = saved_pv;
  if (rc) return rc;
  int kmax = 1;
  for (const auto& st : plan->stages) kmax = std::max(kmax, st.K);
  plan->auto_mfma_min_k = tmf < t32 ? 1 : kmax + 1;
  if (best_ms) *best_ms = best + std::min(t32, tmf);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[arch_name() + "|" + signature(plan)] =
      TuneEntry{bt, bg, plan->auto_mfma_min_k, best_epi, best_grid, bb, bpre ? 1 + plan->prefix_start : 0};
  return CCUT_OK;
}

extern "C" int ccut_autotune_save(const char* path) {
  clear_error();
  if (!path) return fail(CCUT_EINVAL, "path is NULL");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(CCUT_EINVAL, "cannot write %s", path);
  std::fprintf(f, "# ccut autotune cache: key threads grid_cap mfma_min_k epilogue merge_grid block_bits prefix\n");
  for (const auto& kv : g_tune)
    std::fprintf(f, "%s %d %d %d %d %d %d %d\n", kv.first.c_str(), kv.second.threads, kv.second.grid_cap,
                 kv.second.mfma_min_k, kv.second.epilogue, kv.second.merge_grid, kv.second.block_bits,
                 kv.second.prefix);
  std::fclose(f);
  return CCUT_OK;
}

extern "C" int ccut_autotune_load(const char* path) {
  clear_error();
  if (!path) return fail(CCUT_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(CCUT_EINVAL, "cannot read %s", path);
  char key[1024];
  int t, c, k, ep, mg, bb, pf;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  char line[1200];
  while (std::fgets(line, sizeof(line), f)) {
    if (line[0] == '#') continue;
    if (std::sscanf(line, "%1023s %d %d %d %d %d %d %d", key, &t, &c, &k, &ep, &mg, &bb, &pf) == 8 &&
        (t == 256 || t == 512 || t == 1024) && c >= 0 && k >= -1 && ep >= 0 && ep < MERGE_VARIANTS && mg >= 0 &&
        (bb == 0 || (bb > 4 && bb <= PASS_MAX_B)) && pf >= -1 && pf <= 1 + CCUT_MAX_CUTS_PER_SEG)
      g_tune[key] = TuneEntry{t, c, k, ep, mg, bb, pf};
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
  if (int rc = ccut_plan_prepare(plan)) return rc;  // tables must not be copied inside the graph
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* G = new (std::nothrow) ccut_graph();
  if (!G) return fail(CCUT_ENOMEM, "host allocation failed");
  CCUT_HIP(hipGetDevice(&G->device));
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    delete G;
    return hip_fail(e, "hipStreamBeginCapture");
  }
  int rc = ccut_simulate_subcircuits(plan, d_arena, arena_bytes, stream);
  if (rc == 0) rc = ccut_merge_full_state(plan, d_arena, arena_bytes, d_psi, psi_bytes, precision, stream);
  std::string msg = rc ? ccut_last_error() : "";
  e = hipStreamEndCapture(s, &G->graph);
  if (rc || e != hipSuccess) {
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
    return rc ? fail(rc, "%s", msg.c_str()) : hip_fail(e, "hipStreamEndCapture");
  }
  e = hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(G->graph);
    delete G;
    return hip_fail(e, "hipGraphInstantiate");
  }
  *out = G;
  return CCUT_OK;
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
  delete g;
}
