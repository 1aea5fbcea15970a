// Float64 reductions over a complex64 state: |psi|^2, |ref|^2, <ref|psi> and
// max |psi - ref|.  Cutting reproduces the uncut state exactly up to rounding
// (Sec. III of the paper); these numbers measure how closely a computed state
// does.  Two deterministic passes: fixed per-block partials, then one block.
// The max keeps squared distances (the square root, monotone, is taken once).
#include <mutex>

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

__device__ __forceinline__ void accumulate(double v[5], float px_, float py_, float rx_, float ry_) {
  const double px = px_, py = py_, rx = rx_, ry = ry_;
  v[0] += px * px + py * py;
  v[1] += rx * rx + ry * ry;
  v[2] += rx * px + ry * py;
  v[3] += rx * py - ry * px;
  const double dx = px - rx, dy = py - ry;
  v[4] = fmax(v[4], dx * dx + dy * dy);  // squared: one square root at the end
}

// VEC: 16-byte loads (two amplitudes per lane), four of them in flight per array.
template <bool VEC>
__global__ __launch_bounds__(RT) void k_reduce_partial(const float2* __restrict__ psi,
                                                       const float2* __restrict__ ref, uint64_t n,
                                                       double* __restrict__ partials) {
  __shared__ double red[RT / 64 * 5];
  double v[5] = {0, 0, 0, 0, 0};
  const uint64_t stride = (uint64_t)gridDim.x * RT;
  uint64_t i = (uint64_t)blockIdx.x * RT + threadIdx.x;
  if (VEC) {
    const float4* p4 = reinterpret_cast<const float4*>(psi);
    const float4* r4 = reinterpret_cast<const float4*>(ref);
    const uint64_t n4 = n / 2;
    for (; i + 3 * stride < n4; i += 4 * stride) {
      float4 p[4], r[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        p[u] = p4[i + u * stride];
        r[u] = ref ? r4[i + u * stride] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        accumulate(v, p[u].x, p[u].y, r[u].x, r[u].y);
        accumulate(v, p[u].z, p[u].w, r[u].z, r[u].w);
      }
    }
    for (; i < n4; i += stride) {
      const float4 p = p4[i];
      const float4 r = ref ? r4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
      accumulate(v, p.x, p.y, r.x, r.y);
      accumulate(v, p.z, p.w, r.z, r.w);
    }
  } else {
    for (; i < n; i += stride) {
      const float2 p = psi[i];
      const float2 r = ref ? ref[i] : make_float2(0.f, 0.f);
      accumulate(v, p.x, p.y, r.x, r.y);
    }
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
  if (threadIdx.x == 0) {
    for (int i = 0; i < 4; ++i) out[i] = v[i];
    out[4] = sqrt(v[4]);
  }
}

}  // namespace

// ------------------------------------------------ allocation-free variant
// The partials of ccut_norm_fidelity_noalloc live in this fixed array instead of a
// buffer the library allocates: RED_BLOCKS blocks x 5 partials (40 KiB), enough for
// every state size since the partial pass never uses more blocks.  Each device holds
// its own copy at its own address until the process ends.  In host code `scratch`
// names a host-side stand-in, never the device memory: kernels get the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[RED_BLOCKS * 5];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[MAX_DEVICES] = {};
}  // namespace

int reduce_scratch(double** out, uint64_t* n_doubles) {
  int dev = 0;
  CCUT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(CCUT_EUNSUPPORTED, "device id %d", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(CCUT_EHIP, "hipGetSymbolAddress(scratch) returned NULL on device %d", dev);
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  *n_doubles = (uint64_t)RED_BLOCKS * 5;
  return 0;
}

int launch_reduce(const float* psi, const float* ref, uint64_t n, double* d_partials, int n_blocks,
                  double* d_out, hipStream_t s) {
  ProfScope prof(PROF_REDUCE, s);
  const bool vec = (n % 2) == 0 && ((reinterpret_cast<uintptr_t>(psi) | reinterpret_cast<uintptr_t>(ref)) & 15) == 0;
  if (vec)
    hipLaunchKernelGGL(k_reduce_partial<true>, dim3(n_blocks), dim3(RT), 0, s, reinterpret_cast<const float2*>(psi),
                       reinterpret_cast<const float2*>(ref), n, d_partials);
  else
    hipLaunchKernelGGL(k_reduce_partial<false>, dim3(n_blocks), dim3(RT), 0, s, reinterpret_cast<const float2*>(psi),
                       reinterpret_cast<const float2*>(ref), n, d_partials);
  CCUT_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RT), 0, s, d_partials, n_blocks, d_out);
  CCUT_HIP(hipGetLastError());
  return 0;
}

}  // namespace ccut
