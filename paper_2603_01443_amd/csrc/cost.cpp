// Cost model entry points: the closed-form thresholds of Sec. IV, the learned
// MLP (train / predict / gradient) and the cut-or-not decision built on them.
#include <cmath>
#include <mutex>

#include "mlp.h"

namespace ccut {

namespace {

// N_sub = sum_i 2^{c_i}, c_i = cuts on the boundaries next to segment i (Sec. III.A, k = 2).
double n_sub(int n, const int* cb) {
  double s = 0;
  for (int i = 0; i < n; ++i) {
    int ci = (i > 0 ? cb[i - 1] : 0) + (i + 1 < n ? cb[i] : 0);
    s += std::ldexp(1.0, ci);
  }
  return s;
}

// c_total over n-1 boundaries, as even as possible, extras on the lower boundaries.
void split_even(int c_total, int n, int* cb) {
  const int nb = n - 1;
  for (int b = 0; b < nb; ++b) cb[b] = c_total / nb + (b < c_total % nb ? 1 : 0);
}

// Network inputs: the four problem parameters, centred and scaled, then the cost terms of
// Table I for equal blocks (largest segment q_max = ceil(q / n)) and cuts spread evenly over
// the boundaries: log2 N_sub, q_max, log2 (N_sub 2^{q_max} d) for the subcircuit stage and
// log2 (K 2^q) with K = 2^{c_total} terms for the merge.  Uncut rows: n = 1, c_total = 0,
// N_sub = 1, q_max = q (the sub term is then the uncut simulation's 2^q d).
void features(int q, int d, int n, int c_total, float out[MLP_IN]) {
  const double ld = std::log2((double)d);
  double lsub = 0.0;
  int qmax = q;
  if (n >= 2) {
    int cb[CCUT_MAX_SEG];
    split_even(c_total, n, cb);
    lsub = std::log2(n_sub(n, cb));
    qmax = (q + n - 1) / n;
  }
  out[0] = (float)((q - 24.0) / 8.0);
  out[1] = (float)(ld - std::log2(20.0));
  out[2] = (float)(n - 3.0);
  out[3] = (float)((c_total - 4.0) / 4.0);
  out[4] = (float)((lsub - 6.0) / 4.0);
  out[5] = (float)((qmax - 12.0) / 4.0);
  out[6] = (float)((lsub + qmax + ld - 24.0) / 6.0);
  out[7] = (float)((c_total + q - 30.0) / 6.0);
}

std::mutex g_dec_mu;
float* g_dec_buf[64] = {nullptr};

}  // namespace

}  // namespace ccut

using namespace ccut;

extern "C" int ccut_threshold_ctotal(int32_t q, int32_t n, double* bound) {
  clear_error();
  if (!bound || n < 2 || q < 1) return fail(CCUT_EINVAL, "need n >= 2, q >= 1");
  // Eq. (threshold_n2): c_total < q/2.  Eq. (threshold_nge3): slope (n-1)^2/(2n), delta (n-1) log2(n/(n-2)) / 2.
  if (n == 2) *bound = q / 2.0;
  else *bound = q * (n - 1.0) * (n - 1.0) / (2.0 * n) + (n - 1.0) * std::log2((double)n / (n - 2.0)) / 2.0;
  return CCUT_OK;
}

extern "C" int ccut_speedup_margin(int32_t q, int32_t n, const int32_t* cuts_per_boundary, double* margin) {
  clear_error();
  if (!margin || n < 2 || n > CCUT_MAX_SEG || q < n || !cuts_per_boundary) return fail(CCUT_EINVAL, "bad argument");
  int cb[CCUT_MAX_SEG];
  for (int b = 0; b + 1 < n; ++b) {
    if (cuts_per_boundary[b] < 0 || cuts_per_boundary[b] > 1000) return fail(CCUT_EINVAL, "bad cut count");
    cb[b] = cuts_per_boundary[b];
  }
  // Eq. (speedup_depth_free): N_sub / n < 2^{q (1 - 1/n)}; margin in log2 units.
  *margin = q * (1.0 - 1.0 / n) - std::log2(n_sub(n, cb) / n);
  return CCUT_OK;
}

extern "C" int ccut_cost_features(int32_t q, int32_t d, int32_t n, int32_t c_total, float out[8]) {
  clear_error();
  if (!out || q < 1 || d < 1 || n < 1 || n > CCUT_MAX_SEG || c_total < 0) return fail(CCUT_EINVAL, "bad argument");
  features(q, d, n, c_total, out);
  return CCUT_OK;
}

extern "C" int ccut_mlp_work_bytes(int64_t rows, int32_t epochs, uint64_t* bytes) {
  clear_error();
  if (!bytes || rows < 1 || epochs < 0) return fail(CCUT_EINVAL, "bad argument");
  *bytes = mlp_work_floats(rows, epochs) * sizeof(float);
  return CCUT_OK;
}

extern "C" int ccut_mlp_predict(const float* d_params, const float* d_x, int64_t rows, float* d_y, void* stream) {
  clear_error();
  if (!d_params || !d_x || !d_y || rows < 0) return fail(CCUT_EINVAL, "bad argument");
  return mlp_forward(d_params, d_x, rows, d_y, static_cast<hipStream_t>(stream));
}

extern "C" int ccut_mlp_grad(const float* d_params, const float* d_x, const float* d_t, int64_t rows, void* d_work,
                             uint64_t work_bytes, float* d_grad, float* loss, void* stream) {
  clear_error();
  if (!d_params || !d_x || !d_t || !d_work || !d_grad || !loss || rows < 1) return fail(CCUT_EINVAL, "bad argument");
  if (work_bytes < mlp_work_floats(rows, 1) * sizeof(float)) return fail(CCUT_ENOSPC, "work buffer too small");
  return mlp_grad(d_params, d_x, d_t, rows, static_cast<float*>(d_work), d_grad, loss,
                  static_cast<hipStream_t>(stream));
}

extern "C" int ccut_mlp_train(float* d_params, const float* d_x, const float* d_t, int64_t rows, int32_t epochs,
                              float lr, void* d_work, uint64_t work_bytes, float* losses, void* stream) {
  clear_error();
  if (!d_params || !d_x || !d_t || !d_work || rows < 1 || epochs < 0 || !(lr > 0.f))
    return fail(CCUT_EINVAL, "bad argument");
  if (work_bytes < mlp_work_floats(rows, epochs) * sizeof(float)) return fail(CCUT_ENOSPC, "work buffer too small");
  return mlp_train(d_params, d_x, d_t, rows, epochs, lr, static_cast<float*>(d_work), losses, 50,
                   static_cast<hipStream_t>(stream));
}

namespace {
// Closed-form rule: the n whose Eq. (speedup_depth_free) margin is largest and positive, else 0.
int closed_form_choice(int q, int c_total) {
  int best = 0;
  double best_m = 0.0;
  for (int n = 2; n <= 4; ++n) {
    if (n > q) continue;
    int cb[CCUT_MAX_SEG];
    split_even(c_total, n, cb);
    const double m = q * (1.0 - 1.0 / n) - std::log2(n_sub(n, cb) / n);
    if (m > best_m) { best = n; best_m = m; }
  }
  return best;
}
}  // namespace

extern "C" int ccut_decide(int32_t q, int32_t d, int32_t c_total, const float* d_params, double budget_s,
                           double margin, int32_t* choice, double* predicted_s, void* stream) {
  clear_error();
  if (!choice || q < 1 || d < 1 || c_total < 0 || !(margin >= 0.0 && margin < 1.0))
    return fail(CCUT_EINVAL, "bad argument");
  const int cands[4] = {1, 2, 3, 4};
  const int cf = closed_form_choice(q, c_total);
  if (!d_params) {
    *choice = cf;
    if (predicted_s) *predicted_s = NAN;
    return CCUT_OK;
  }
  // Learned model: argmin of predicted wall clock over {uncut, n = 2, 3, 4}.
  float x[4 * MLP_IN];
  int valid[4];
  for (int i = 0; i < 4; ++i) {
    const int n = cands[i];
    valid[i] = n <= q;
    features(q, d, n, n == 1 ? 0 : c_total, x + MLP_IN * i);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  CCUT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(CCUT_EUNSUPPORTED, "device id %d", dev);
  std::lock_guard<std::mutex> lk(g_dec_mu);
  if (!g_dec_buf[dev]) CCUT_HIP(hipMalloc((void**)&g_dec_buf[dev], 64 * sizeof(float)));
  float* dx = g_dec_buf[dev];
  float* dy = dx + 4 * MLP_IN;  // 4 x MLP_IN inputs, then 4 x 3 outputs (<= 64 floats)
  static_assert(4 * MLP_IN + 12 <= 64, "decision buffer");
  CCUT_HIP(hipMemcpyAsync(dx, x, sizeof(x), hipMemcpyHostToDevice, s));
  if (int rc = mlp_forward(d_params, dx, 4, dy, s)) return rc;
  float y[12];
  CCUT_HIP(hipMemcpyAsync(y, dy, sizeof(y), hipMemcpyDeviceToHost, s));
  CCUT_HIP(hipStreamSynchronize(s));
  int best = -1;
  double best_t = INFINITY, t_cf = INFINITY;
  for (int i = 0; i < 4; ++i) {
    if (!valid[i]) continue;
    const double t = cands[i] == 1 ? std::exp((double)y[3 * i + 1])
                                   : std::exp((double)y[3 * i]) + std::exp((double)y[3 * i + 1]) +
                                         std::exp((double)y[3 * i + 2]);
    if (t < best_t) { best_t = t; best = cands[i]; }
    if ((cands[i] == 1 ? 0 : cands[i]) == cf) t_cf = t;
  }
  // guard: leave the closed-form choice only for a predicted gain of more than `margin`
  if ((best == 1 ? 0 : best) != cf && best_t > (1.0 - margin) * t_cf) {
    best = cf == 0 ? 1 : cf;
    best_t = t_cf;
  }
  *choice = best == 1 ? 0 : best;
  if (budget_s > 0 && best_t > budget_s) *choice = -1;  // nothing fits the budget
  if (predicted_s) *predicted_s = best_t;
  return CCUT_OK;
}
