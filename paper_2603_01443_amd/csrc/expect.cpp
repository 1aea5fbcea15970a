// Pauli-string expectation values of the cut state from the subcircuit states
// (no merge): per-segment matrices G_i on the GPU, then the contraction over
// the cut bits in float64 on the host, boundary by boundary:
//   E_0[u][u']  = W_0[u][u'] G_0[u][u']
//   E_i[v][v']  = W_i[v][v'] sum_{u,u'} E_{i-1}[u][u'] G_i[u + 2^{c_{i-1}} v][u' + 2^{c_{i-1}} v']
//   <O>         = sum_{u,u'} E_{n-2}[u][u'] G_{n-1}[u][u']
// with W_b[u][u'] = conj(w_b(u)) w_b(u'), where w_b(u) is the product of the
// term weights of boundary b's cuts (s_0 = 1/(1+i), s_1 = i/(1+i) for CZ / CX,
// Eq. CZ; the Schmidt coefficients for the other kinds) and segment i's variant index
// r = (lower-boundary bits) + 2^{c_{i-1}} (upper-boundary bits).
#include <complex>
#include <cstring>
#include <vector>

#include "plan.h"

using namespace ccut;

namespace {

// Workspace: the summed V x V matrices of all segments first (one contiguous
// region, copied to the host at once), then each segment's per-split partials.
struct WorkLayout {
  std::vector<uint64_t> fin_off, part_off;
  std::vector<GramShape> shape;
  uint64_t fin_bytes = 0, total = 0;
};

WorkLayout work_layout(const ccut_plan* P) {
  WorkLayout w;
  uint64_t off = 0;
  for (const auto& S : P->segs) {
    const uint64_t V = (uint64_t)1 << S.c;
    w.fin_off.push_back(off);
    off = align256(off + V * V * sizeof(double2));
  }
  w.fin_bytes = off;
  for (const auto& S : P->segs) {
    const uint64_t V = (uint64_t)1 << S.c;
    const GramShape g = gram_shape((int)V, (uint64_t)1 << S.q);
    const int sp = g.splits;
    w.shape.push_back(g);
    w.part_off.push_back(off);
    off = align256(off + (uint64_t)sp * V * V * sizeof(double2));
  }
  w.total = off;
  return w;
}

// W_b[u][u'] = conj(w_b(u)) w_b(u'), w_b = the weights of boundary b's term combinations
std::vector<cd> boundary_weights(const ccut_plan* P, int b) {
  const auto& w = P->bw[b];
  const size_t V = w.size();
  std::vector<cd> out(V * V);
  for (size_t u = 0; u < V; ++u)
    for (size_t v = 0; v < V; ++v) out[u * V + v] = std::conj(w[u]) * w[v];
  return out;
}

}  // namespace

extern "C" int ccut_expectation_work_bytes(const ccut_plan_t* plan, uint64_t* bytes) {
  clear_error();
  if (!plan || !bytes) return fail(CCUT_EINVAL, "NULL argument");
  *bytes = work_layout(plan).total;
  return CCUT_OK;
}

extern "C" int ccut_expectation_pauli(ccut_plan_t* plan, const void* d_arena, uint64_t arena_bytes,
                                      const char* pauli, void* d_work, uint64_t work_bytes_in, double out[2],
                                      void* stream) {
  clear_error();
  if (!plan || !d_arena || !pauli || !d_work || !out) return fail(CCUT_EINVAL, "NULL argument");
  if (arena_bytes < plan->state_bytes) return fail(CCUT_ENOSPC, "arena smaller than the plan's states");
  if (std::strlen(pauli) != (size_t)plan->q)
    return fail(CCUT_EINVAL, "Pauli label has %zu characters for q=%d", std::strlen(pauli), plan->q);
  for (int j = 0; j < plan->q; ++j)
    if (!std::strchr("IXYZ", pauli[j]) || pauli[j] == 0)
      return fail(CCUT_EINVAL, "Pauli label character %d is '%c' (I, X, Y or Z)", j, pauli[j]);
  for (const auto& S : plan->segs)
    if (S.c > CCUT_MAX_EXPECT_CUTS)
      return fail(CCUT_EUNSUPPORTED, "expectation values need at most %d cuts per segment", CCUT_MAX_EXPECT_CUTS);
  const WorkLayout wl = work_layout(plan);
  if (work_bytes_in < wl.total)
    return fail(CCUT_ENOSPC, "work buffer has %llu bytes, needs %llu", (unsigned long long)work_bytes_in,
                (unsigned long long)wl.total);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const char* base = static_cast<const char*>(d_arena);
  char* work = static_cast<char*>(d_work);
  std::vector<cd> phase(plan->n_seg);
  for (int i = 0; i < plan->n_seg; ++i) {
    const auto& S = plan->segs[i];
    uint32_t flip = 0, zy = 0;
    int ny = 0;
    for (int t = 0; t < S.q; ++t) {
      const char p = pauli[S.off + t];
      if (p == 'X' || p == 'Y') flip |= 1u << t;
      if (p == 'Z' || p == 'Y') zy |= 1u << t;
      ny += p == 'Y';
    }
    cd ph = 1.0;
    for (int k = 0; k < ny; ++k) ph *= cd(0, -1);  // Y = -i Z X on each Y qubit
    phase[i] = ph;
    if (int rc = launch_gram(reinterpret_cast<const float2*>(base + S.arena_off), 1 << S.c, (uint64_t)1 << S.q, flip,
                             zy, wl.shape[i], reinterpret_cast<double2*>(work + wl.part_off[i]),
                             reinterpret_cast<double2*>(work + wl.fin_off[i]), s))
      return rc;
  }
  std::lock_guard<std::mutex> lock(plan->expect_mu);
  if (plan->expect_host_bytes < wl.fin_bytes) {
    if (plan->expect_host) (void)hipHostFree(plan->expect_host);
    plan->expect_host = nullptr;
    plan->expect_host_bytes = 0;
    CCUT_HIP(hipHostMalloc(&plan->expect_host, wl.fin_bytes, hipHostMallocDefault));
    plan->expect_host_bytes = wl.fin_bytes;
  }
  CCUT_HIP(hipMemcpyAsync(plan->expect_host, work, wl.fin_bytes, hipMemcpyDeviceToHost, s));
  CCUT_HIP(hipStreamSynchronize(s));
  // per-segment G with the Y phase
  std::vector<std::vector<cd>> G(plan->n_seg);
  for (int i = 0; i < plan->n_seg; ++i) {
    const int64_t V = (int64_t)1 << plan->segs[i].c;
    const double2* p = reinterpret_cast<const double2*>(static_cast<const char*>(plan->expect_host) + wl.fin_off[i]);
    G[i].resize((size_t)(V * V));
    for (int64_t e = 0; e < V * V; ++e) G[i][(size_t)e] = cd(p[e].x, p[e].y) * phase[i];
  }
  cd result;
  const int n = plan->n_seg;
  if (n == 1) {
    result = G[0][0];
  } else {
    int cprev = plan->c_b[0];
    int64_t U = (int64_t)1 << cprev;
    std::vector<cd> E = boundary_weights(plan, 0);
    for (int64_t e = 0; e < U * U; ++e) E[(size_t)e] *= G[0][(size_t)e];
    for (int i = 1; i + 1 < n; ++i) {
      const int cnext = plan->c_b[i];
      const int64_t Vn = (int64_t)1 << cnext, Vi = U * Vn;
      std::vector<cd> W = boundary_weights(plan, i), En((size_t)(Vn * Vn), cd(0));
      for (int64_t v = 0; v < Vn; ++v)
        for (int64_t vp = 0; vp < Vn; ++vp) {
          cd acc = 0.0;
          for (int64_t u = 0; u < U; ++u)
            for (int64_t up = 0; up < U; ++up)
              acc += E[(size_t)(u * U + up)] * G[i][(size_t)((u + U * v) * Vi + (up + U * vp))];
          En[(size_t)(v * Vn + vp)] = W[(size_t)(v * Vn + vp)] * acc;
        }
      E.swap(En);
      U = Vn;
    }
    cd acc = 0.0;
    for (int64_t e = 0; e < U * U; ++e) acc += E[(size_t)e] * G[n - 1][(size_t)e];
    result = acc;
  }
  out[0] = result.real();
  out[1] = result.imag();
  return CCUT_OK;
}
