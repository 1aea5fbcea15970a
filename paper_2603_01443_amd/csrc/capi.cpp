// C-ABI entry points: error reporting, device tables, and the device stages
// of the pipeline (subcircuit simulation, merge, uncut baseline, diagnostics).
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>

#include "merge_mfma.h"
#include "plan.h"

namespace ccut {

// Term count from which CCUT_PREC_AUTO merges on MFMA.
constexpr int MFMA_MIN_TERMS = 8;

namespace {
thread_local char g_err[512] = "";
}

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_err[0] = 0; }

int hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? CCUT_ENOMEM : CCUT_EHIP, "%s failed: %s", what, hipGetErrorString(e));
}

void release_device(DeviceTables& t) {
  if (t.device < 0) return;
  int cur = 0;
  if (hipGetDevice(&cur) == hipSuccess && cur != t.device) (void)hipSetDevice(t.device);
  if (t.blob) (void)hipFree(t.blob);
  if (cur != t.device) (void)hipSetDevice(cur);
  t = DeviceTables();
}

namespace {
uint64_t pad256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

template <class T>
void pack(std::vector<unsigned char>& img, const std::vector<T>& v, uint64_t& off) {
  off = img.size();
  const uint64_t bytes = v.size() * sizeof(T);
  img.resize(pad256(off + bytes));
  if (bytes) std::memcpy(img.data() + off, v.data(), bytes);
}

// Pinned staging ring: host images are copied into a slot, and the slot's
// event (recorded after the device copy) gates its reuse.
constexpr int RING_SLOTS = 32;
constexpr uint64_t SLOT_BYTES = 256 << 10;
struct StagingRing {
  unsigned char* host = nullptr;
  hipEvent_t ev[RING_SLOTS] = {};
  bool used[RING_SLOTS] = {};
  int next = 0;
};
std::mutex g_ring_mu;
StagingRing g_ring[64];
}  // namespace

void pack_image(ccut_plan* P) {
  P->image.clear();
  pack(P->image, P->kops, P->img_ops);
  pack(P->image, P->pass_descs, P->img_passes);
  pack(P->image, P->stage_descs, P->img_stages);
  pack(P->image, P->jobs, P->img_jobs);
  pack(P->image, P->weights, P->img_weights);
  pack(P->image, P->grefs, P->img_grefs);
  if (P->image.empty()) P->image.resize(256);
  P->image_gen++;
}

int staged_copy(void* dst, const void* src, uint64_t bytes, hipStream_t s) {
  if (bytes > SLOT_BYTES) {  // large images go directly (may wait for the stream)
    CCUT_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    return 0;
  }
  int dev = 0;
  CCUT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(CCUT_EUNSUPPORTED, "device id %d", dev);
  std::lock_guard<std::mutex> lk(g_ring_mu);
  StagingRing& R = g_ring[dev];
  if (!R.host) {
    CCUT_HIP(hipHostMalloc((void**)&R.host, SLOT_BYTES * RING_SLOTS, hipHostMallocDefault));
    for (int i = 0; i < RING_SLOTS; ++i) CCUT_HIP(hipEventCreateWithFlags(&R.ev[i], hipEventDisableTiming));
  }
  const int slot = R.next;
  R.next = (R.next + 1) % RING_SLOTS;
  if (R.used[slot]) CCUT_HIP(hipEventSynchronize(R.ev[slot]));
  unsigned char* h = R.host + (uint64_t)slot * SLOT_BYTES;
  std::memcpy(h, src, bytes);
  // a kernel reading the pinned slot starts sooner than a copy-engine transfer
  void* hd = nullptr;
  if ((bytes & 15) == 0 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0 &&
      hipHostGetDevicePointer(&hd, h, 0) == hipSuccess && hd) {
    if (int rc = launch_table_copy(dst, hd, bytes, s)) return rc;
  } else {
    (void)hipGetLastError();  // a failed device-pointer query leaves an error behind
    CCUT_HIP(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, s));
  }
  CCUT_HIP(hipEventRecord(R.ev[slot], s));
  R.used[slot] = true;
  return 0;
}

// Copies a table image to a new device allocation (synchronous).
int upload_tables(DeviceTables& t, const std::vector<unsigned char>& img, uint64_t o_ops, uint64_t o_pass,
                  uint64_t o_stage, uint64_t o_jobs, uint64_t o_w, uint64_t o_grefs) {
  int dev = 0;
  CCUT_HIP(hipGetDevice(&dev));
  if (t.device == dev) return 0;
  release_device(t);
  void* blob = nullptr;
  CCUT_HIP(hipMalloc(&blob, img.size()));
  hipError_t e = hipMemcpy(blob, img.data(), img.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(blob);
    return hip_fail(e, "table upload");
  }
  unsigned char* b = static_cast<unsigned char*>(blob);
  t.blob = blob;
  t.ops = reinterpret_cast<KOp*>(b + o_ops);
  t.passes = reinterpret_cast<PassDesc*>(b + o_pass);
  t.stages = reinterpret_cast<StageDesc*>(b + o_stage);
  t.jobs = reinterpret_cast<SimJob*>(b + o_jobs);
  t.weights = reinterpret_cast<float*>(b + o_w);
  t.grefs = reinterpret_cast<GroupRef*>(b + o_grefs);
  t.device = dev;
  return 0;
}

// Device addresses of a plan's tables for a call on `arena`: the plan-owned
// copy when prepared on this device, otherwise a fresh copy into the arena.
// Device addresses of the plan's tables: its own copy after ccut_plan_prepare, else
// the arena's table region, which receives the image (through the staging ring)
// unless `reuse` is set and the last copy went to this arena from the current
// image build.  The merge reuses: the arena it reads holds this plan's states,
// so the simulation call that wrote them also left the tables there.
int plan_tables(ccut_plan* P, char* arena, hipStream_t s, DeviceTables& out, bool reuse) {
  int dev = 0;
  CCUT_HIP(hipGetDevice(&dev));
  if (P->dev.device == dev) {
    out = DeviceTables();
    out.ops = P->dev.ops;
    out.passes = P->dev.passes;
    out.stages = P->dev.stages;
    out.jobs = P->dev.jobs;
    out.weights = P->dev.weights;
    out.grefs = P->dev.grefs;
    return 0;
  }
  unsigned char* b = reinterpret_cast<unsigned char*>(arena + P->tables_off);
  if (!(reuse && P->staged_arena == arena && P->staged_gen == P->image_gen)) {
    if (int rc = staged_copy(b, P->image.data(), P->image.size(), s)) return rc;
    P->staged_arena = arena;
    P->staged_gen = P->image_gen;
  }
  out = DeviceTables();
  out.ops = reinterpret_cast<KOp*>(b + P->img_ops);
  out.passes = reinterpret_cast<PassDesc*>(b + P->img_passes);
  out.stages = reinterpret_cast<StageDesc*>(b + P->img_stages);
  out.jobs = reinterpret_cast<SimJob*>(b + P->img_jobs);
  out.weights = reinterpret_cast<float*>(b + P->img_weights);
  out.grefs = reinterpret_cast<GroupRef*>(b + P->img_grefs);
  return 0;
}

// Per-device buffer for reduction partials (allocated once, kept for the process).
static std::mutex g_red_mu;
static double* g_red_buf[64] = {nullptr};

int reduction_buffer(double** out) {
  int dev = 0;
  CCUT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(CCUT_EUNSUPPORTED, "device id %d", dev);
  static std::mutex alloc_mu;
  std::lock_guard<std::mutex> lk(alloc_mu);
  if (!g_red_buf[dev]) CCUT_HIP(hipMalloc((void**)&g_red_buf[dev], (RED_BLOCKS * 5 + 8) * sizeof(double)));
  *out = g_red_buf[dev];
  return 0;
}

// ---------------------------------------------------------------- uncut cache
// Uncut passes use 2^13-amplitude blocks and 512-thread workgroups (16 amplitudes
// per thread, two workgroups per CU by LDS).  Measured at q = 28, d = 20 over
// blocks of 2^12 .. 2^14 and 256 .. 1024 threads: 45.8 ms, against 49.8 ms for the
// best 2^14 configuration (one workgroup per CU, so every stage barrier idles it).
constexpr int UNCUT_BLOCK_BITS = 13;
constexpr int UNCUT_THREADS = 512;

struct UncutProg {
  uint64_t key = 0;
  int32_t q = 0;
  std::vector<ccut_gate_t> gates;
  std::vector<PassDesc> descs;
  std::vector<StageDesc> stages;
  std::vector<KOp> kops;
  std::vector<SimJob> jobs;  // one per pass
  std::vector<GroupRef> grefs;
  DeviceTables dev;
  uint4* gtab = nullptr;     // MFMA group tables (built once)
  uint64_t stamp = 0;
};

void release_uncut(UncutProg& U) {
  if (U.gtab && U.dev.device >= 0) {
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != U.dev.device) (void)hipSetDevice(U.dev.device);
    (void)hipFree(U.gtab);
    if (cur != U.dev.device) (void)hipSetDevice(cur);
  }
  U.gtab = nullptr;
  release_device(U.dev);
}

static std::mutex g_uncut_mu;
static std::map<uint64_t, std::unique_ptr<UncutProg>> g_uncut;
static uint64_t g_uncut_clock = 0;
constexpr size_t UNCUT_CACHE = 8;

static uint64_t fnv1a(const void* p, size_t n, uint64_t h) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
  return h;
}

int compile_uncut(int32_t q, const ccut_gate_t* gates, int64_t n_gates, UncutProg& U) {
  ProgramBuilder pb(q);
  for (int64_t k = 0; k < n_gates; ++k) {
    const ccut_gate_t& g = gates[k];
    if (int rc = check_gate(g, q, k)) return rc;
    pb.gate(g, 0);
  }
  std::vector<Pass> passes;
  if (int rc = schedule_passes(pb.prog, UNCUT_BLOCK_BITS, 4, passes, true, true)) return rc;
  for (const Pass& p : passes) {
    int pid = append_pass(p, q, U.descs, U.stages, U.kops, U.grefs, true);  // tables built once per program
    SimJob j;
    std::memset(&j, 0, sizeof(j));
    j.pass_id = pid;
    U.jobs.push_back(j);
  }
  return 0;
}

}  // namespace ccut

using namespace ccut;

extern "C" const char* ccut_last_error(void) { return g_err; }

extern "C" const char* ccut_version(void) { return "ccut 0.1 gfx950"; }

extern "C" int ccut_plan_prepare(ccut_plan_t* plan) {
  clear_error();
  if (!plan) return fail(CCUT_EINVAL, "plan is NULL");
  return upload_tables(plan->dev, plan->image, plan->img_ops, plan->img_passes, plan->img_stages, plan->img_jobs,
                       plan->img_weights, plan->img_grefs);
}

extern "C" int ccut_simulate_subcircuits(ccut_plan_t* plan, void* d_arena, uint64_t arena_bytes, void* stream) {
  clear_error();
  if (!plan || !d_arena) return fail(CCUT_EINVAL, "NULL argument");
  if (arena_bytes < plan->sim_bytes)
    return fail(CCUT_ENOSPC, "arena has %llu bytes, the simulation needs %llu", (unsigned long long)arena_bytes,
                (unsigned long long)plan->sim_bytes);
  hipStream_t s = static_cast<hipStream_t>(stream);
  DeviceTables T;
  if (int rc = plan_tables(plan, static_cast<char*>(d_arena), s, T, false)) return rc;
  const uint4* gtab = nullptr;
  if (plan->sim_precision == CCUT_SIM_FP16X3 && !plan->grefs.empty()) {
    uint4* g = reinterpret_cast<uint4*>(static_cast<char*>(d_arena) + plan->gtab_off);
    if (int rc = launch_group_tables(T.ops, T.grefs, (int)plan->grefs.size(), g, s)) return rc;
    gtab = g;
  }
  for (const auto& L : plan->launches) {
    if (plan->sim_per_variant) {
      for (int j = 0; j < L.n_jobs; ++j) {
        const SimJob& job = plan->jobs[L.job_begin + j];
        const int nb = plan->pass_descs[job.pass_id].n_blocks;
        if (int rc = launch_sim(T.jobs + L.job_begin, L.n_jobs, nb, job.wg_begin, T.passes, T.stages, T.ops, gtab,
                                static_cast<float*>(d_arena), plan->bmax, L.rec_cap, plan->sim_threads,
                                0, s))
          return rc;
      }
      continue;
    }
    if (int rc = launch_sim(T.jobs + L.job_begin, L.n_jobs, L.total_wg, 0, T.passes, T.stages, T.ops, gtab,
                            static_cast<float*>(d_arena), plan->bmax, L.rec_cap, plan->sim_threads,
                            plan->sim_grid_cap, s))
      return rc;
  }
  return CCUT_OK;
}

extern "C" int ccut_merge_full_state(ccut_plan_t* plan, void* d_arena, uint64_t arena_bytes, void* d_psi,
                                     uint64_t psi_bytes, int32_t precision, void* stream) {
  clear_error();
  if (!plan || !d_arena || !d_psi) return fail(CCUT_EINVAL, "NULL argument");
  if (!plan->merge_ok)
    return fail(CCUT_EUNSUPPORTED, "q=%d: the merged state exceeds one GPU (q <= %d); expectation values "
                "need no merge", plan->q, CCUT_MAX_Q);
  if (arena_bytes < plan->total_arena) return fail(CCUT_ENOSPC, "arena too small");
  if (psi_bytes < plan->psi_bytes)
    return fail(CCUT_ENOSPC, "psi has %llu bytes, needs %llu", (unsigned long long)psi_bytes,
                (unsigned long long)plan->psi_bytes);
  if (precision < CCUT_PREC_AUTO || precision > CCUT_PREC_FP16X2)
    return fail(CCUT_EINVAL, "unknown precision %d", precision);
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* arena = static_cast<char*>(d_arena);
  DeviceTables T;
  if (int rc = plan_tables(plan, arena, s, T, true)) return rc;
  if (plan->n_seg == 1) {
    CCUT_HIP(hipMemcpyAsync(d_psi, arena + plan->segs[0].arena_off, plan->psi_bytes, hipMemcpyDeviceToDevice, s));
    return CCUT_OK;
  }
  auto buf = [&](int id) -> float* {
    if (id == 0) return reinterpret_cast<float*>(arena);
    if (id == 1) return reinterpret_cast<float*>(arena + plan->temp_off[0]);
    if (id == 2) return reinterpret_cast<float*>(arena + plan->temp_off[1]);
    return static_cast<float*>(d_psi);
  };
  for (const MergeStage& st : plan->stages) {
    int mode = precision;
    if (mode == CCUT_PREC_AUTO) {
      const int kmin = plan->auto_mfma_min_k >= 0 ? plan->auto_mfma_min_k : MFMA_MIN_TERMS;
      mode = st.K >= kmin ? plan->auto_mfma_mode : CCUT_PREC_FP32;
    }
    if (mode == CCUT_PREC_FP32 || !merge_mfma_supported(st.qx, st.qy)) {
      // shapes below one MFMA tile take the float32 kernel, which is at least as accurate
      if (int rc = launch_merge_f32(st, buf(st.a_src), buf(st.b_src), buf(st.out_dst), T.weights, s))
        return rc;
      continue;
    }
    MergeMfmaArgs a;
    a.A = reinterpret_cast<const float2*>(buf(st.a_src)) + st.a_off;
    a.a_kstride = st.a_kstride;
    a.a_bstride = st.a_bstride;
    a.B = reinterpret_cast<const float2*>(buf(st.b_src)) + st.b_off;
    a.b_kstride = st.b_kstride;
    a.b_bstride = st.b_bstride;
    a.w = reinterpret_cast<const float2*>(T.weights) + st.weight_off;
    a.K = st.K;
    a.qx = st.qx;
    a.qy = st.qy;
    a.S = mfma_steps(st.K);
    a.batch = st.batch;
    a.r_batch = st.a_bstride ? st.batch : 1;
    a.l_plane_stride = mfma_l_plane(st.qy, a.S);
    a.r_plane_stride = mfma_r_plane(st.qx, a.S);
    uint4* ws = reinterpret_cast<uint4*>(arena + plan->split_off);
    a.Lhi = ws;
    a.Llo = a.Lhi + (uint64_t)a.batch * a.l_plane_stride;
    a.Rhi = a.Llo + (uint64_t)a.batch * a.l_plane_stride;
    a.Rlo = a.Rhi + (uint64_t)a.r_batch * a.r_plane_stride;
    a.out = buf(st.out_dst) + 2 * st.out_off;
    a.out_bstride = st.out_bstride;
    if (int rc = launch_merge_mfma(a, mode, plan->merge_epilogue, plan->merge_grid_cap, s)) return rc;
  }
  return CCUT_OK;
}

extern "C" int ccut_simulate_uncut(int32_t q, const ccut_gate_t* gates, int64_t n_gates, void* d_psi,
                                   uint64_t psi_bytes, void* stream) {
  clear_error();
  if (q < 1 || q > CCUT_MAX_Q) return fail(CCUT_EINVAL, "q=%d outside [1, %d]", q, CCUT_MAX_Q);
  if (!d_psi || n_gates < 0 || (n_gates > 0 && !gates)) return fail(CCUT_EINVAL, "bad argument");
  if (psi_bytes < ((uint64_t)8 << q)) return fail(CCUT_ENOSPC, "psi buffer too small for q=%d", q);
  uint64_t key = fnv1a(&q, sizeof(q), 1469598103934665603ull);
  key = fnv1a(gates, sizeof(ccut_gate_t) * (size_t)n_gates, key);
  int dev = 0;
  CCUT_HIP(hipGetDevice(&dev));
  key = fnv1a(&dev, sizeof(dev), key);
  std::lock_guard<std::mutex> lk(g_uncut_mu);
  UncutProg* U = nullptr;
  auto it = g_uncut.find(key);
  if (it != g_uncut.end() && it->second->q == q && it->second->gates.size() == (size_t)n_gates &&
      std::memcmp(it->second->gates.data(), gates, sizeof(ccut_gate_t) * (size_t)n_gates) == 0) {
    U = it->second.get();
  } else {
    auto fresh = std::make_unique<UncutProg>();
    fresh->key = key;
    fresh->q = q;
    fresh->gates.assign(gates, gates + n_gates);
    if (int rc = compile_uncut(q, gates, n_gates, *fresh)) return rc;
    std::vector<unsigned char> img;
    uint64_t o_ops, o_pass, o_stage, o_jobs, o_w, o_g;
    pack(img, fresh->kops, o_ops);
    pack(img, fresh->descs, o_pass);
    pack(img, fresh->stages, o_stage);
    pack(img, fresh->jobs, o_jobs);
    pack(img, fresh->grefs, o_g);
    o_w = img.size();
    if (int rc = upload_tables(fresh->dev, img, o_ops, o_pass, o_stage, o_jobs, o_w, o_g)) return rc;
    if (!fresh->grefs.empty()) {  // operand tables built once, before the program is first used
      hipError_t e = hipMalloc((void**)&fresh->gtab, fresh->grefs.size() * GROUP_TABLE_UINT4 * sizeof(uint4));
      if (e != hipSuccess) {
        fresh->gtab = nullptr;
        release_uncut(*fresh);
        return hip_fail(e, "group table allocation");
      }
      int rc = launch_group_tables(fresh->dev.ops, fresh->dev.grefs, (int)fresh->grefs.size(), fresh->gtab, nullptr);
      if (rc == 0 && (e = hipDeviceSynchronize()) != hipSuccess) rc = hip_fail(e, "group table build");
      if (rc) {
        release_uncut(*fresh);
        return rc;
      }
    }
    if (g_uncut.size() >= UNCUT_CACHE) {
      auto oldest = g_uncut.begin();
      for (auto i = g_uncut.begin(); i != g_uncut.end(); ++i)
        if (i->second->stamp < oldest->second->stamp) oldest = i;
      release_uncut(*oldest->second);
      g_uncut.erase(oldest);
    }
    U = fresh.get();
    g_uncut[key] = std::move(fresh);
  }
  U->stamp = ++g_uncut_clock;
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (size_t p = 0; p < U->jobs.size(); ++p) {
    const PassDesc& d = U->descs[p];
    if (int rc = launch_sim(U->dev.jobs + p, 1, d.n_blocks, 0, U->dev.passes, U->dev.stages, U->dev.ops, U->gtab,
                            static_cast<float*>(d_psi), UNCUT_BLOCK_BITS,
                            d.stage_count > 0 ? d.op_count + d.stage_count : 0, UNCUT_THREADS, 0, s))
      return rc;
  }
  return CCUT_OK;
}

extern "C" int ccut_norm_fidelity(const void* d_psi, const void* d_ref, int32_t q, double out[5], void* stream) {
  clear_error();
  if (!d_psi || !out) return fail(CCUT_EINVAL, "NULL argument");
  if (q < 0 || q > CCUT_MAX_Q) return fail(CCUT_EINVAL, "q=%d out of range", q);
  double* buf = nullptr;
  if (int rc = reduction_buffer(&buf)) return rc;
  std::lock_guard<std::mutex> lk(g_red_mu);  // one partials buffer per device
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t n = (uint64_t)1 << q;
  int blocks = (int)std::min<uint64_t>(RED_BLOCKS, (n + 255) / 256);
  if (int rc = launch_reduce(static_cast<const float*>(d_psi), static_cast<const float*>(d_ref), n, buf, blocks,
                             buf + RED_BLOCKS * 5, s))
    return rc;
  CCUT_HIP(hipMemcpyAsync(out, buf + RED_BLOCKS * 5, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
  CCUT_HIP(hipStreamSynchronize(s));
  return CCUT_OK;
}

extern "C" int ccut_norm_fidelity_noalloc(const void* d_psi, const void* d_ref, int32_t q, double* d_out,
                                          void* stream) {
  clear_error();
  if (!d_psi || !d_out) return fail(CCUT_EINVAL, "NULL argument");
  if (q < 0 || q > CCUT_MAX_Q)
    return fail(CCUT_EINVAL, "q=%d outside [0, %d]: the fixed scratch array covers states up to 2^%d amplitudes", q,
                CCUT_MAX_Q, CCUT_MAX_Q);
  double* scratch = nullptr;
  uint64_t cap = 0;
  if (int rc = reduce_scratch(&scratch, &cap)) return rc;
  const uint64_t n = (uint64_t)1 << q;
  const int blocks = (int)std::min<uint64_t>(RED_BLOCKS, (n + 255) / 256);
  if ((uint64_t)blocks * 5 > cap)
    return fail(CCUT_ENOSPC, "%d reduction blocks need %d doubles of scratch, the array holds %llu", blocks,
                blocks * 5, (unsigned long long)cap);
  // every partial the final pass reads is written by this call's first pass: nothing to clear
  return launch_reduce(static_cast<const float*>(d_psi), static_cast<const float*>(d_ref), n, scratch, blocks,
                       d_out, static_cast<hipStream_t>(stream));
}
