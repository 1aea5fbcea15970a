// Merging (Algorithm 3 of the paper) with float32 vector arithmetic.
//
// One stage computes, for every batch entry beta,
//   out[beta][y * NX + x] = sum_k w_k A(beta, k)[x] B(beta, k)[y],
// i.e. the sum of weighted Kronecker products psi_B^(k) (x) psi_A^(k) with the
// A factor on the low qubits.  Each thread owns one column x and RB rows: its
// A values stream through registers once per k while the B values of the
// workgroup's rows are uniform across the wavefront (scalar loads when a
// whole workgroup shares its rows).  Every output amplitude is written once,
// with consecutive lanes on consecutive addresses.
#include "ccut_internal.h"

namespace ccut {

namespace {

constexpr int MT = 256;

struct MergeArgs {
  const float2* A;
  const float2* B;
  float2* out;
  const float2* w;
  uint64_t a_kstride, a_bstride, b_kstride, b_bstride, out_bstride;
  int K, qx, qy;
};

template <int RB>
__global__ __launch_bounds__(MT) void k_merge_f32(MergeArgs a) {
  const int NX = 1 << a.qx, NY = 1 << a.qy;
  const int TX = NX < MT ? NX : MT;
  const int GY = MT / TX;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int x = blockIdx.x * TX + tx;
  const int y0 = (blockIdx.y * GY + ty) * RB;
  const int beta = blockIdx.z;
  if (y0 >= NY) return;
  const float2* A = a.A + beta * a.a_bstride + x;
  const float2* B = a.B + beta * a.b_bstride + y0;
  float2 acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = make_float2(0.f, 0.f);
  const int nr = (NY - y0) < RB ? (NY - y0) : RB;
  for (int k = 0; k < a.K; ++k) {
    const float2 wk = a.w[k];
    const float2 av = A[(uint64_t)k * a.a_kstride];
    const float2 ak = make_float2(wk.x * av.x - wk.y * av.y, wk.x * av.y + wk.y * av.x);
    const float2* Bk = B + (uint64_t)k * a.b_kstride;
    if (nr == RB) {
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const float2 bv = Bk[r];
        acc[r].x = fmaf(ak.x, bv.x, fmaf(-ak.y, bv.y, acc[r].x));
        acc[r].y = fmaf(ak.x, bv.y, fmaf(ak.y, bv.x, acc[r].y));
      }
    } else {
      for (int r = 0; r < nr; ++r) {
        const float2 bv = Bk[r];
        acc[r].x = fmaf(ak.x, bv.x, fmaf(-ak.y, bv.y, acc[r].x));
        acc[r].y = fmaf(ak.x, bv.y, fmaf(ak.y, bv.x, acc[r].y));
      }
    }
  }
  float2* o = a.out + beta * a.out_bstride + (uint64_t)y0 * NX + x;
  if (nr == RB) {
#pragma unroll
    for (int r = 0; r < RB; ++r) o[(uint64_t)r * NX] = acc[r];
  } else {
    for (int r = 0; r < nr; ++r) o[(uint64_t)r * NX] = acc[r];
  }
}

}  // namespace

int launch_merge_f32(const MergeStage& st, const float* A, const float* B, float* out, const float* d_weights,
                     hipStream_t s) {
  constexpr int RB = 16;
  MergeArgs a;
  a.A = reinterpret_cast<const float2*>(A) + st.a_off;
  a.B = reinterpret_cast<const float2*>(B) + st.b_off;
  a.out = reinterpret_cast<float2*>(out) + st.out_off;
  a.w = reinterpret_cast<const float2*>(d_weights) + st.weight_off;
  a.a_kstride = st.a_kstride;
  a.a_bstride = st.a_bstride;
  a.b_kstride = st.b_kstride;
  a.b_bstride = st.b_bstride;
  a.out_bstride = st.out_bstride;
  a.K = st.K;
  a.qx = st.qx;
  a.qy = st.qy;
  const int NX = 1 << st.qx, NY = 1 << st.qy;
  const int TX = NX < MT ? NX : MT;
  const int GY = MT / TX;
  const int rows_per_wg = GY * RB;
  dim3 grid((NX + TX - 1) / TX, (NY + rows_per_wg - 1) / rows_per_wg, st.batch);
  if (grid.y > 65535u || grid.z > 65535u) return fail(CCUT_EUNSUPPORTED, "merge grid too large");
  hipLaunchKernelGGL(k_merge_f32<RB>, grid, dim3(MT), 0, s, a);
  CCUT_HIP(hipGetLastError());
  return 0;
}

}  // namespace ccut
