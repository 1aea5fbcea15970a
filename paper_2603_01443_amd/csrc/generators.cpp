// Seeded circuit generators of the C-ABI: the random brickwork used for the
// measured workloads (the problem statement of Sec. IV: q qubits, depth d, n
// contiguous segments, c_b cuts on boundary b) and the paper's own staircase
// family (Fig. 1).  Input data only: nothing here belongs to the cutting
// method.  The recipe is fixed so that independent implementations (the
// Python generator the tests use) produce the same gate list bit for bit.
#include <cstring>
#include <vector>

#include "ccut_internal.h"

namespace ccut {
namespace {

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the state advances by the
// golden gamma; the output is the two-round xor-shift-multiply finaliser.
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  // double in [0, 1) from the top 53 bits
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

constexpr double kTwoPi = 2.0 * 3.14159265358979323846;

ccut_gate_t make_gate(int kind, int q0, int q1, double p0, double p1) {
  ccut_gate_t g;
  std::memset(&g, 0, sizeof(g));
  g.kind = kind;
  g.q0 = q0;
  g.q1 = q1;
  g.p0 = p0;
  g.p1 = p1;
  return g;
}

int copy_out(const std::vector<ccut_gate_t>& gates, ccut_gate_t* out, int64_t cap, int64_t* n_out) {
  *n_out = (int64_t)gates.size();
  if (!out) return CCUT_OK;  // size query
  if (cap < (int64_t)gates.size())
    return fail(CCUT_ENOSPC, "gate buffer holds %lld gates, %zu needed", (long long)cap, gates.size());
  std::memcpy(out, gates.data(), gates.size() * sizeof(ccut_gate_t));
  return CCUT_OK;
}

}  // namespace
}  // namespace ccut

using namespace ccut;

extern "C" int ccut_brickwork(int32_t q, int32_t d, int32_t n_seg, int32_t c_total, const int32_t* seg_sizes,
                              const int32_t* cuts_per_boundary, uint64_t seed, ccut_gate_t* out, int64_t cap,
                              int64_t* n_out) {
  clear_error();
  if (!n_out) return fail(CCUT_EINVAL, "n_out is NULL");
  if (q < 1 || q > 62 || d < 0 || n_seg < 1 || n_seg > CCUT_MAX_SEG || n_seg > q || c_total < 0)
    return fail(CCUT_EINVAL, "bad brickwork shape q=%d d=%d n=%d c_total=%d", q, d, n_seg, c_total);
  // segment sizes: given, or floor(q / n) with the remainder on the last segments
  std::vector<int> sizes(n_seg);
  int sum = 0;
  for (int i = 0; i < n_seg; ++i) {
    sizes[i] = seg_sizes ? seg_sizes[i] : q / n_seg + (i >= n_seg - q % n_seg ? 1 : 0);
    if (sizes[i] < 1) return fail(CCUT_EINVAL, "segment %d has size %d", i, sizes[i]);
    sum += sizes[i];
  }
  if (sum != q) return fail(CCUT_EINVAL, "segment sizes sum to %d, not q = %d", sum, q);
  // cuts per boundary: given, or as even as possible with the extras on the lower boundaries
  const int nb = n_seg - 1;
  std::vector<int> cb(nb);
  int csum = 0;
  for (int b = 0; b < nb; ++b) {
    cb[b] = cuts_per_boundary ? cuts_per_boundary[b] : c_total / nb + (b < c_total % nb ? 1 : 0);
    if (cb[b] < 0) return fail(CCUT_EINVAL, "boundary %d has %d cuts", b, cb[b]);
    if (cb[b] > d) return fail(CCUT_EINVAL, "boundary %d: at most one cut per layer (c_b <= d)", b);
    csum += cb[b];
  }
  if (csum != c_total) return fail(CCUT_EINVAL, "cuts per boundary sum to %d, not c_total = %d", csum, c_total);
  // boundary b sits between qubits beta_b - 1 and beta_b
  std::vector<int> beta(nb);
  for (int b = 0, acc = 0; b < nb; ++b) beta[b] = acc += sizes[b];
  std::vector<char> boundary_pair(q, 0);  // pair (i, i + 1) crosses a boundary
  for (int b = 0; b < nb; ++b) boundary_pair[beta[b] - 1] = 1;
  // cut layers of boundary b: floor(j d / c_b), j = 0 .. c_b - 1 (distinct since c_b <= d)
  std::vector<std::vector<char>> cut_layer(nb, std::vector<char>(d, 0));
  for (int b = 0; b < nb; ++b)
    for (int j = 0; j < cb[b]; ++j) cut_layer[b][(int64_t)j * d / cb[b]] = 1;

  SplitMix64 rng{seed};
  std::vector<ccut_gate_t> gates;
  gates.reserve((size_t)d * (q + q / 2 + nb));
  for (int layer = 0; layer < d; ++layer) {
    for (int j = 0; j < q; ++j) {
      const double theta = kTwoPi * rng.uniform();
      const double phi = kTwoPi * rng.uniform();
      gates.push_back(make_gate(CCUT_GATE_RYRZ, j, -1, theta, phi));
    }
    for (int i = layer % 2; i < q - 1; i += 2)
      if (!boundary_pair[i]) gates.push_back(make_gate(CCUT_GATE_CZ, i, i + 1, 0.0, 0.0));
    for (int b = 0; b < nb; ++b)
      if (cut_layer[b][layer]) gates.push_back(make_gate(CCUT_GATE_CZ, beta[b] - 1, beta[b], 0.0, 0.0));
  }
  return copy_out(gates, out, cap, n_out);
}

extern "C" int ccut_staircase(int32_t q, int32_t copies, int32_t tx_layers, ccut_gate_t* out, int64_t cap,
                              int64_t* n_out) {
  clear_error();
  if (!n_out) return fail(CCUT_EINVAL, "n_out is NULL");
  if (q < 2 || q > 62 || copies < 1 || tx_layers < 0)
    return fail(CCUT_EINVAL, "bad staircase shape q=%d copies=%d tx_layers=%d", q, copies, tx_layers);
  std::vector<ccut_gate_t> gates;
  for (int j = 0; j < q; ++j) gates.push_back(make_gate(CCUT_GATE_H, j, -1, 0.0, 0.0));
  for (int t = 0; t < tx_layers; ++t) {
    gates.push_back(make_gate(CCUT_GATE_T, 0, -1, 0.0, 0.0));
    gates.push_back(make_gate(CCUT_GATE_X, 0, -1, 0.0, 0.0));
  }
  for (int c = 0; c < copies; ++c)
    for (int i = 0; i < q - 1; ++i) {
      if (i == 0) gates.push_back(make_gate(CCUT_GATE_T, 0, -1, 0.0, 0.0));
      gates.push_back(make_gate(CCUT_GATE_T, i + 1, -1, 0.0, 0.0));
      gates.push_back(make_gate(CCUT_GATE_CX, i, i + 1, 0.0, 0.0));
      gates.push_back(make_gate(CCUT_GATE_T, i, -1, 0.0, 0.0));
      gates.push_back(make_gate(CCUT_GATE_T, i + 1, -1, 0.0, 0.0));
    }
  for (int t = 0; t < tx_layers; ++t) {
    gates.push_back(make_gate(CCUT_GATE_T, q - 1, -1, 0.0, 0.0));
    gates.push_back(make_gate(CCUT_GATE_X, q - 1, -1, 0.0, 0.0));
  }
  return copy_out(gates, out, cap, n_out);
}
