// Merging (Algorithm 3 of the paper) with float32 vector arithmetic.
//
// One stage computes, for every batch entry beta,
//   out[beta][y * NX + x] = sum_k w_k A(beta, k)[x] B(beta, k)[y],
// the sum of weighted Kronecker products psi_B^(k) (x) psi_A^(k) with the A
// factor on the low qubits.  Each thread owns one column x and RB rows.  The
// workgroup stages the B values of its rows for a chunk of KC terms in LDS
// (read back as wavefront-wide broadcasts) and each thread keeps the KC
// weighted A values of its column in registers, so the inner loop is pure
// FMA.  Every output amplitude is written once, consecutive lanes on
// consecutive addresses.  From 128 columns on, each thread owns two adjacent
// columns (k_merge_f32_wide, 16-byte stores); columns narrower than 64 use a
// plain loop.
#include "ccut_internal.h"

namespace ccut {

namespace {

typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int MT = 256;
constexpr int RB = 16;
constexpr int KC = 16;

struct MergeArgs {
  const float2* A;
  const float2* B;
  float2* out;
  const float2* w;
  uint64_t a_kstride, a_bstride, b_kstride, b_bstride, out_bstride;
  int K, qx, qy;
};

__device__ __forceinline__ void cfma(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x));
  acc.y = fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y));
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// NX >= 64: TX = min(NX, 256) columns, GY = 256 / TX row groups of RB rows.
__global__ __launch_bounds__(MT) void k_merge_f32_tiled(MergeArgs a) {
  __shared__ float2 Bs[KC * (MT / 64) * RB];
  const int NX = 1 << a.qx, NY = 1 << a.qy;
  const int TX = NX < MT ? NX : MT;
  const int GY = MT / TX;
  const int TY = GY * RB;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int ny_tiles = (NY + TY - 1) / TY;  // tiles are flattened into grid.x
  const int x = (blockIdx.x / ny_tiles) * TX + tx;
  const int y0 = (blockIdx.x % ny_tiles) * TY;
  const int beta = blockIdx.z;
  const float2* A = a.A + beta * a.a_bstride + x;
  const float2* B = a.B + beta * a.b_bstride + y0;
  float2 acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = make_float2(0.f, 0.f);
  for (int k0 = 0; k0 < a.K; k0 += KC) {
    const int kn = (a.K - k0) < KC ? (a.K - k0) : KC;
    __syncthreads();
    for (int i = threadIdx.x; i < KC * TY; i += MT) {
      const int kk = i / TY, row = i % TY;
      float2 v = make_float2(0.f, 0.f);
      if (kk < kn && y0 + row < NY) v = B[(uint64_t)(k0 + kk) * a.b_kstride + row];
      Bs[i] = v;
    }
    __syncthreads();
    float2 av[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
      av[kk] = kk < kn ? cmul(a.w[k0 + kk], A[(uint64_t)(k0 + kk) * a.a_kstride]) : make_float2(0.f, 0.f);
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const float2* bk = Bs + kk * TY + ty * RB;
#pragma unroll
      for (int r = 0; r < RB; ++r) cfma(acc[r], av[kk], bk[r]);
    }
  }
  const int yb = y0 + ty * RB;
  float2* o = a.out + beta * a.out_bstride + (uint64_t)yb * NX + x;
#pragma unroll
  for (int r = 0; r < RB; ++r)
    if (yb + r < NY) o[(uint64_t)r * NX] = acc[r];
}

// NX >= 128: as k_merge_f32_tiled, but every thread owns two adjacent columns, so that
// each lane stores 16 bytes (a wavefront writes 1 KiB of a row per instruction, with
// non-temporal stores: the output is not read again here).  TX = min(NX, 512) columns
// per tile row, GY = 256 / (TX / 2) row groups of RB rows.  Same summation order per
// amplitude as k_merge_f32_tiled.  Terms come in chunks of min(K, 16) (K is a power of
// two), so that a small K runs no zero terms.  A workgroup sweeps several row tiles of
// its column tile; with a single chunk (K <= 16) it loads its weighted A values once.
template <int KCW>  // terms per chunk: min(K, KC), so that small K does no zero terms
__global__ __launch_bounds__(MT) void k_merge_f32_wide(MergeArgs a, int row_tiles_per_wg) {
  constexpr int KC = KCW;
  __shared__ float2 Bs[KC * (MT / 64) * RB];
  const int NX = 1 << a.qx, NY = 1 << a.qy;
  const int TX = NX < 2 * MT ? NX : 2 * MT;
  const int TT = TX / 2;
  const int GY = MT / TT;
  const int TY = GY * RB;
  const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
  const int ny_tiles = (NY + TY - 1) / TY;
  const int ny_groups = (ny_tiles + row_tiles_per_wg - 1) / row_tiles_per_wg;
  const int x = (blockIdx.x / ny_groups) * TX + 2 * tx;
  const int rt0 = (blockIdx.x % ny_groups) * row_tiles_per_wg;
  const int beta = blockIdx.z;
  const float4* A = reinterpret_cast<const float4*>(a.A + beta * a.a_bstride + x);
  const uint64_t a_k4 = a.a_kstride / 2;  // float4 stride between terms
  const bool one_chunk = a.K <= KC;       // then the weighted A values are loaded once
  float2 av0[KC], av1[KC];
  for (int rt = rt0; rt < rt0 + row_tiles_per_wg && rt < ny_tiles; ++rt) {
    const int y0 = rt * TY;
    const float2* B = a.B + beta * a.b_bstride + y0;
    float2 acc0[RB], acc1[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc0[r] = acc1[r] = make_float2(0.f, 0.f);
    for (int k0 = 0; k0 < a.K; k0 += KC) {
      const int kn = (a.K - k0) < KC ? (a.K - k0) : KC;
      __syncthreads();
      for (int i = threadIdx.x; i < KC * TY; i += MT) {
        const int kk = i / TY, row = i % TY;
        float2 v = make_float2(0.f, 0.f);
        if (kk < kn && y0 + row < NY) v = B[(uint64_t)(k0 + kk) * a.b_kstride + row];
        Bs[i] = v;
      }
      if (!one_chunk || rt == rt0) {
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
          if (kk < kn) {
            const float4 v = A[(uint64_t)(k0 + kk) * a_k4];
            const float2 w = a.w[k0 + kk];
            av0[kk] = cmul(w, make_float2(v.x, v.y));
            av1[kk] = cmul(w, make_float2(v.z, v.w));
          } else {
            av0[kk] = av1[kk] = make_float2(0.f, 0.f);
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        const float2* bk = Bs + kk * TY + ty * RB;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const float2 b = bk[r];
          cfma(acc0[r], av0[kk], b);
          cfma(acc1[r], av1[kk], b);
        }
      }
    }
    const int yb = y0 + ty * RB;
    f32x4* o = reinterpret_cast<f32x4*>(a.out + beta * a.out_bstride + (uint64_t)yb * NX + x);
    const uint64_t o_row = (uint64_t)NX / 2;
#pragma unroll
    for (int r = 0; r < RB; ++r)
      if (yb + r < NY) {
        const f32x4 v = {acc0[r].x, acc0[r].y, acc1[r].x, acc1[r].y};
        __builtin_nontemporal_store(v, o + (uint64_t)r * o_row);
      }
  }
}

// NX < 64: one thread per (x, row group), plain loop over terms.
__global__ __launch_bounds__(MT) void k_merge_f32_small(MergeArgs a) {
  const int NX = 1 << a.qx, NY = 1 << a.qy;
  const uint64_t id = (uint64_t)blockIdx.x * MT + threadIdx.x;
  const uint64_t total = (uint64_t)NX * NY;
  const int beta = blockIdx.z;
  if (id >= total) return;
  const uint64_t x = id % NX, y = id / NX;
  float2 acc = make_float2(0.f, 0.f);
  for (int k = 0; k < a.K; ++k) {
    const float2 av = cmul(a.w[k], a.A[beta * a.a_bstride + (uint64_t)k * a.a_kstride + x]);
    cfma(acc, av, a.B[beta * a.b_bstride + (uint64_t)k * a.b_kstride + y]);
  }
  a.out[beta * a.out_bstride + y * NX + x] = acc;
}

}  // namespace

int launch_merge_f32(const MergeStage& st, const float* A, const float* B, float* out, const float* d_weights,
                     hipStream_t s) {
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
  if (st.batch > 65535) return fail(CCUT_EUNSUPPORTED, "merge batch too large");
  const uint64_t NX = (uint64_t)1 << st.qx, NY = (uint64_t)1 << st.qy;
  const bool aligned = ((reinterpret_cast<uintptr_t>(a.A) | reinterpret_cast<uintptr_t>(a.out)) & 15) == 0 &&
                       (a.a_kstride % 2) == 0 && (a.a_bstride % 2) == 0 && (a.out_bstride % 2) == 0;
  if (NX >= 2 * 64 && aligned) {
    const uint64_t TX = NX < 2 * MT ? NX : 2 * MT;
    const uint64_t TY = (MT / (TX / 2)) * RB;
    const uint64_t ny_tiles = (NY + TY - 1) / TY;
    // several row tiles per workgroup while the grid stays above ~16 workgroups per CU
    int per = 1;
    while (per < 8 && (ny_tiles / (2 * per)) * (NX / TX) * st.batch >= 4096) per *= 2;
    const uint64_t tiles = ((ny_tiles + per - 1) / per) * (NX / TX);
    if (tiles > 0x7fffffffu) return fail(CCUT_EUNSUPPORTED, "merge grid too large");
    dim3 grid((unsigned)tiles, 1, st.batch);
    ProfScope prof(PROF_MERGE_F32, s);
    if (st.K >= 16) hipLaunchKernelGGL(k_merge_f32_wide<16>, grid, dim3(MT), 0, s, a, per);
    else if (st.K >= 8) hipLaunchKernelGGL(k_merge_f32_wide<8>, grid, dim3(MT), 0, s, a, per);
    else if (st.K >= 4) hipLaunchKernelGGL(k_merge_f32_wide<4>, grid, dim3(MT), 0, s, a, per);
    else if (st.K >= 2) hipLaunchKernelGGL(k_merge_f32_wide<2>, grid, dim3(MT), 0, s, a, per);
    else hipLaunchKernelGGL(k_merge_f32_wide<1>, grid, dim3(MT), 0, s, a, per);
  } else if (NX >= 64) {
    const uint64_t TX = NX < MT ? NX : MT;
    const uint64_t TY = (MT / TX) * RB;
    const uint64_t tiles = ((NY + TY - 1) / TY) * (NX / TX);
    if (tiles > 0x7fffffffu) return fail(CCUT_EUNSUPPORTED, "merge grid too large");
    dim3 grid((unsigned)tiles, 1, st.batch);
    ProfScope prof(PROF_MERGE_F32, s);
    hipLaunchKernelGGL(k_merge_f32_tiled, grid, dim3(MT), 0, s, a);
  } else {
    const uint64_t blocks = (NX * NY + MT - 1) / MT;
    if (blocks > 0x7fffffffu) return fail(CCUT_EUNSUPPORTED, "merge grid too large");
    ProfScope prof(PROF_MERGE_F32, s);
    hipLaunchKernelGGL(k_merge_f32_small, dim3((unsigned)blocks, 1, st.batch), dim3(MT), 0, s, a);
  }
  CCUT_HIP(hipGetLastError());
  return 0;
}

}  // namespace ccut
