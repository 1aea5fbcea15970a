// Float64 reductions over a complex64 state: |psi|^2, |ref|^2, <ref|psi> and
// max |psi - ref|.  Cutting reproduces the uncut state exactly up to rounding
// (Sec. III of the paper); these numbers measure how closely a computed state
// does.  Two deterministic passes: fixed per-block partials, then one block.
#include "ccut_internal.h"

namespace ccut {

namespace {

constexpr int RT = 256;

__device__ __forceinline__ void block_sum5(double v[5], double* red) {
  // wavefront reduction, then across the 4 wavefronts of the block
  for (int i = 0; i < 4; ++i)
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off);
  for (int off = 32; off > 0; off >>= 1) v[4] = fmax(v[4], __shfl_xor(v[4], off));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
    for (int i = 0; i < 5; ++i) red[wid * 5 + i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < RT / 64; ++w) {
      for (int i = 0; i < 4; ++i) v[i] += red[w * 5 + i];
      v[4] = fmax(v[4], red[w * 5 + 4]);
    }
  }
}

__global__ __launch_bounds__(RT) void k_reduce_partial(const float2* __restrict__ psi,
                                                       const float2* __restrict__ ref, uint64_t n,
                                                       double* __restrict__ partials) {
  __shared__ double red[RT / 64 * 5];
  double v[5] = {0, 0, 0, 0, 0};
  const uint64_t stride = (uint64_t)gridDim.x * RT;
  for (uint64_t i = (uint64_t)blockIdx.x * RT + threadIdx.x; i < n; i += stride) {
    const float2 p = psi[i];
    const float2 r = ref ? ref[i] : make_float2(0.f, 0.f);
    const double px = p.x, py = p.y, rx = r.x, ry = r.y;
    v[0] += px * px + py * py;
    v[1] += rx * rx + ry * ry;
    v[2] += rx * px + ry * py;
    v[3] += rx * py - ry * px;
    const double dx = px - rx, dy = py - ry;
    v[4] = fmax(v[4], sqrt(dx * dx + dy * dy));
  }
  block_sum5(v, red);
  if (threadIdx.x == 0)
    for (int i = 0; i < 5; ++i) partials[(uint64_t)blockIdx.x * 5 + i] = v[i];
}

__global__ __launch_bounds__(RT) void k_reduce_final(const double* __restrict__ partials, int nparts,
                                                     double* __restrict__ out) {
  __shared__ double red[RT / 64 * 5];
  double v[5] = {0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < nparts; i += RT) {
    for (int j = 0; j < 4; ++j) v[j] += partials[(uint64_t)i * 5 + j];
    v[4] = fmax(v[4], partials[(uint64_t)i * 5 + 4]);
  }
  block_sum5(v, red);
  if (threadIdx.x == 0)
    for (int i = 0; i < 5; ++i) out[i] = v[i];
}

}  // namespace

int launch_reduce(const float* psi, const float* ref, uint64_t n, double* d_partials, int n_blocks,
                  double* d_out, hipStream_t s) {
  ProfScope prof(PROF_REDUCE, s);
  hipLaunchKernelGGL(k_reduce_partial, dim3(n_blocks), dim3(RT), 0, s, reinterpret_cast<const float2*>(psi),
                     reinterpret_cast<const float2*>(ref), n, d_partials);
  CCUT_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RT), 0, s, d_partials, n_blocks, d_out);
  CCUT_HIP(hipGetLastError());
  return 0;
}

}  // namespace ccut
