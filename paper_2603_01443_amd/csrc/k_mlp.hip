// Learned cost model: an 8-64-64-3 tanh MLP trained full-batch with Adam,
// hand-written for gfx950.  It maps features of (q, d, n, c_total) to the
// natural log of the three stage times of the paper's Eq. (runtime_decomp)
// (T_pre, T_sub, T_merge); the decision rule built on it is compared with the
// closed-form thresholds of Sec. IV.
//
// Parameter layout (4931 floats): W1[8][64], b1[64], W2[64][64], b2[64],
// W3[64][3], b3[3].  Loss: mean squared error over rows and outputs.
//
// Training step = three kernels:
//   k_mlp_fwd_bwd : a workgroup takes 32 rows, runs forward and backward in
//                   LDS and writes the chunk's parameter gradient and loss;
//   k_mlp_adam    : one thread per parameter sums the chunk gradients in a
//                   fixed order (deterministic) and applies Adam with bias
//                   correction from the device step counter;
//   k_mlp_tick    : advances the step counter and records the epoch loss.
// Keeping the step counter on the device lets a captured HIP graph of several
// epochs be replayed.
#include <cmath>

#include "ccut_internal.h"
#include "mlp.h"

namespace ccut {

namespace {

constexpr int NI = MLP_IN, NH = MLP_HIDDEN, NO = MLP_OUT;
constexpr int OW1 = 0, OB1 = OW1 + NI * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH * NO;
static_assert(OB3 + NO == MLP_PARAMS, "parameter layout");
constexpr int RC = MLP_ROWS_PER_BLOCK;  // rows per workgroup (LDS: ~53 KiB at 32 rows)
constexpr int TPB = 256;

// Forward (and optionally backward) for rows [r0, r0 + RC).
template <bool BACKWARD>
__global__ __launch_bounds__(TPB) void k_mlp_fwd_bwd(const float* __restrict__ P, const float* __restrict__ X,
                                                     const float* __restrict__ T, int64_t rows,
                                                     float* __restrict__ Y, float* __restrict__ part) {
  __shared__ float w[MLP_PARAMS];
  __shared__ float x[RC][NI];
  __shared__ float h1[RC][NH + 1];
  __shared__ float h2[RC][NH + 1];
  __shared__ float g2[RC][NH + 1];  // dL/da2
  __shared__ float g1[RC][NH + 1];  // dL/da1
  __shared__ float gy[RC][NO];
  __shared__ float lsum[TPB / 64];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * RC;
  for (int i = tid; i < MLP_PARAMS; i += TPB) w[i] = P[i];
  for (int i = tid; i < RC * NI; i += TPB) {
    const int r = i / NI, c = i % NI;
    x[r][c] = (r0 + r < rows) ? X[(r0 + r) * NI + c] : 0.f;
  }
  __syncthreads();
  // layer 1
  for (int i = tid; i < RC * NH; i += TPB) {
    const int r = i / NH, j = i % NH;
    float a = w[OB1 + j];
#pragma unroll
    for (int k = 0; k < NI; ++k) a = fmaf(x[r][k], w[OW1 + k * NH + j], a);
    h1[r][j] = tanhf(a);
  }
  __syncthreads();
  // layer 2
  for (int i = tid; i < RC * NH; i += TPB) {
    const int r = i / NH, j = i % NH;
    float a = w[OB2 + j];
    for (int k = 0; k < NH; ++k) a = fmaf(h1[r][k], w[OW2 + k * NH + j], a);
    h2[r][j] = tanhf(a);
  }
  __syncthreads();
  // output layer and loss gradient
  float lacc = 0.f;
  for (int i = tid; i < RC * NO; i += TPB) {
    const int r = i / NO, o = i % NO;
    float a = w[OB3 + o];
    for (int k = 0; k < NH; ++k) a = fmaf(h2[r][k], w[OW3 + k * NO + o], a);
    if (!BACKWARD) {
      if (r0 + r < rows) Y[(r0 + r) * NO + o] = a;
    } else {
      float g = 0.f;
      if (r0 + r < rows) {
        const float d = a - T[(r0 + r) * NO + o];
        lacc += d * d;
        g = 2.f * d / (float)(rows * NO);
      }
      gy[r][o] = g;
    }
  }
  if (!BACKWARD) return;
  for (int off = 32; off > 0; off >>= 1) lacc += __shfl_xor(lacc, off);
  if ((tid & 63) == 0) lsum[tid >> 6] = lacc;
  __syncthreads();
  // dL/da2 = (gy W3^T) * (1 - h2^2)
  for (int i = tid; i < RC * NH; i += TPB) {
    const int r = i / NH, j = i % NH;
    float g = 0.f;
#pragma unroll
    for (int o = 0; o < NO; ++o) g = fmaf(gy[r][o], w[OW3 + j * NO + o], g);
    g2[r][j] = g * (1.f - h2[r][j] * h2[r][j]);
  }
  __syncthreads();
  // dL/da1 = (g2 W2^T) * (1 - h1^2)
  for (int i = tid; i < RC * NH; i += TPB) {
    const int r = i / NH, k = i % NH;
    float g = 0.f;
    for (int j = 0; j < NH; ++j) g = fmaf(g2[r][j], w[OW2 + k * NH + j], g);
    g1[r][k] = g * (1.f - h1[r][k] * h1[r][k]);
  }
  __syncthreads();
  // chunk gradients: sums over the chunk's rows in row order
  float* out = part + (uint64_t)blockIdx.x * MLP_PART_STRIDE;
  for (int p = tid; p < MLP_PARAMS; p += TPB) {
    float g = 0.f;
    if (p < OB1) {
      const int k = p / NH, j = p % NH;
      for (int r = 0; r < RC; ++r) g = fmaf(x[r][k], g1[r][j], g);
    } else if (p < OW2) {
      const int j = p - OB1;
      for (int r = 0; r < RC; ++r) g += g1[r][j];
    } else if (p < OB2) {
      const int k = (p - OW2) / NH, j = (p - OW2) % NH;
      for (int r = 0; r < RC; ++r) g = fmaf(h1[r][k], g2[r][j], g);
    } else if (p < OW3) {
      const int j = p - OB2;
      for (int r = 0; r < RC; ++r) g += g2[r][j];
    } else if (p < OB3) {
      const int k = (p - OW3) / NO, o = (p - OW3) % NO;
      for (int r = 0; r < RC; ++r) g = fmaf(h2[r][k], gy[r][o], g);
    } else {
      const int o = p - OB3;
      for (int r = 0; r < RC; ++r) g += gy[r][o];
    }
    out[p] = g;
  }
  if (tid == 0) {
    float l = 0.f;
    for (int i = 0; i < TPB / 64; ++i) l += lsum[i];
    out[MLP_PARAMS] = l;  // squared error of the chunk
  }
}

// Adam update of every parameter from the summed chunk gradients.
__global__ __launch_bounds__(TPB) void k_mlp_adam(float* __restrict__ P, const float* __restrict__ part,
                                                  int chunks, float* __restrict__ m, float* __restrict__ v,
                                                  const int* __restrict__ step, float lr, float* __restrict__ grad) {
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= MLP_PARAMS) return;
  float g = 0.f;
  for (int c = 0; c < chunks; ++c) g += part[(uint64_t)c * MLP_PART_STRIDE + p];
  if (grad) grad[p] = g;
  if (lr == 0.f) return;  // gradient only
  const int t = *step + 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mm = b1 * m[p] + (1.f - b1) * g;
  const float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float mhat = mm / (1.f - powf(b1, (float)t));
  const float vhat = vv / (1.f - powf(b2, (float)t));
  P[p] -= lr * mhat / (sqrtf(vhat) + eps);
}

// Advances the step counter and stores the epoch's mean squared error.
__global__ void k_mlp_tick(const float* __restrict__ part, int chunks, int64_t rows, int* __restrict__ step,
                           float* __restrict__ losses, int max_epochs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float l = 0.f;
  for (int c = 0; c < chunks; ++c) l += part[(uint64_t)c * MLP_PART_STRIDE + MLP_PARAMS];
  const int t = *step;
  if (t < max_epochs) losses[t] = l / (float)(rows * NO);
  *step = t + 1;
}

__global__ void k_mlp_zero(float* __restrict__ p, uint64_t n, int* __restrict__ step) {
  const uint64_t i = (uint64_t)blockIdx.x * TPB + threadIdx.x;
  if (i < n) p[i] = 0.f;
  if (i == 0) *step = 0;
}

}  // namespace

uint64_t mlp_work_floats(int64_t rows, int epochs) {
  const uint64_t chunks = (uint64_t)((rows + RC - 1) / RC);
  return chunks * MLP_PART_STRIDE + 2 * (uint64_t)MLP_PARAMS + (uint64_t)(epochs > 0 ? epochs : 1) + 64;
}

int mlp_forward(const float* P, const float* X, int64_t rows, float* Y, hipStream_t s) {
  if (rows <= 0) return 0;
  const int chunks = (int)((rows + RC - 1) / RC);
  ProfScope prof(PROF_MLP, s);
  hipLaunchKernelGGL(k_mlp_fwd_bwd<false>, dim3(chunks), dim3(TPB), 0, s, P, X, nullptr, rows, Y, nullptr);
  CCUT_HIP(hipGetLastError());
  return 0;
}

namespace {
struct MlpWork {
  float* part;
  float* m;
  float* v;
  float* losses;
  int* step;
  int chunks;
};
MlpWork carve(float* work, int64_t rows, int epochs) {
  MlpWork w;
  w.chunks = (int)((rows + RC - 1) / RC);
  w.part = work;
  w.m = w.part + (uint64_t)w.chunks * MLP_PART_STRIDE;
  w.v = w.m + MLP_PARAMS;
  w.losses = w.v + MLP_PARAMS;
  w.step = reinterpret_cast<int*>(w.losses + (epochs > 0 ? epochs : 1));
  return w;
}

int one_epoch(float* P, const float* X, const float* T, int64_t rows, const MlpWork& w, float lr, int epochs,
              float* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_fwd_bwd<true>, dim3(w.chunks), dim3(TPB), 0, s, P, X, T, rows, nullptr, w.part);
  CCUT_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_PARAMS + TPB - 1) / TPB), dim3(TPB), 0, s, P, w.part, w.chunks, w.m,
                     w.v, w.step, lr, grad);
  CCUT_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mlp_tick, dim3(1), dim3(64), 0, s, w.part, w.chunks, rows, w.step, w.losses, epochs);
  CCUT_HIP(hipGetLastError());
  return 0;
}
}  // namespace

int mlp_grad(const float* P, const float* X, const float* T, int64_t rows, float* work, float* grad, float* loss,
             hipStream_t s) {
  MlpWork w = carve(work, rows, 1);
  const uint64_t zn = 2 * (uint64_t)MLP_PARAMS + 1;
  hipLaunchKernelGGL(k_mlp_zero, dim3((unsigned)((zn + TPB - 1) / TPB)), dim3(TPB), 0, s, w.m, zn, w.step);
  CCUT_HIP(hipGetLastError());
  ProfScope prof(PROF_MLP, s);
  if (int rc = one_epoch(const_cast<float*>(P), X, T, rows, w, 0.f, 1, grad, s)) return rc;
  CCUT_HIP(hipMemcpyAsync(loss, w.losses, sizeof(float), hipMemcpyDeviceToHost, s));
  CCUT_HIP(hipStreamSynchronize(s));
  return 0;
}

int mlp_train(float* P, const float* X, const float* T, int64_t rows, int epochs, float lr, float* work,
              float* losses_host, int graph_epochs, hipStream_t s) {
  if (epochs <= 0) return 0;
  MlpWork w = carve(work, rows, epochs);
  const uint64_t zn = 2 * (uint64_t)MLP_PARAMS + (uint64_t)epochs;
  hipLaunchKernelGGL(k_mlp_zero, dim3((unsigned)((zn + TPB - 1) / TPB)), dim3(TPB), 0, s, w.m, zn, w.step);
  CCUT_HIP(hipGetLastError());
  ProfScope prof(PROF_MLP, s);
  int done = 0;
  if (graph_epochs > 1 && s != nullptr && epochs >= graph_epochs) {
    // capture graph_epochs epochs once, replay while whole groups remain
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    CCUT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = 0;
    for (int e = 0; e < graph_epochs && rc == 0; ++e) rc = one_epoch(P, X, T, rows, w, lr, epochs, nullptr, s);
    hipError_t ce = hipStreamEndCapture(s, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(ie, "hipGraphInstantiate");
    }
    while (epochs - done >= graph_epochs) {
      hipError_t le = hipGraphLaunch(ge, s);
      if (le != hipSuccess) {
        (void)hipGraphExecDestroy(ge);
        (void)hipGraphDestroy(g);
        return hip_fail(le, "hipGraphLaunch");
      }
      done += graph_epochs;
    }
    CCUT_HIP(hipStreamSynchronize(s));
    (void)hipGraphExecDestroy(ge);
    (void)hipGraphDestroy(g);
  }
  for (; done < epochs; ++done)
    if (int rc = one_epoch(P, X, T, rows, w, lr, epochs, nullptr, s)) return rc;
  if (losses_host) {
    CCUT_HIP(hipMemcpyAsync(losses_host, w.losses, sizeof(float) * (size_t)epochs, hipMemcpyDeviceToHost, s));
  }
  CCUT_HIP(hipStreamSynchronize(s));
  return 0;
}

}  // namespace ccut
