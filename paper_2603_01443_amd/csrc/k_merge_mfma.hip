// Merging (Algorithm 3 of the paper) as a split-precision GEMM on gfx950 MFMA.
//
// One merge stage  Psi[y][x] = sum_k w_k A_k[x] B_k[y]  (complex) is the real GEMM
//   C (M x 2N) = L (M x 2K) . R (2K x 2N),   M = 2^qy rows, N = 2^qx columns,
// with L[y][2k] = Re B_k[y], L[y][2k+1] = Im B_k[y] and, for A'_k = w_k A_k,
//   R[2k][2x] =  Re A'_k[x]   R[2k][2x+1]   = Im A'_k[x]
//   R[2k+1][2x] = -Im A'_k[x] R[2k+1][2x+1] = Re A'_k[x],
// so row y of C is exactly the interleaved complex64 row of Psi (no permute).
//
// Float32 accuracy from 16-bit MFMA inputs: every factor value v is split into
// hi = round16(v) and lo = round16(v - hi), and C = Lhi.Rhi + Lhi.Rlo + Llo.Rhi
// with float32 accumulation (the lo.lo term, ~2^-16 relative for bfloat16, is
// dropped).  For float16 both factors are scaled by 2^14 first so that lo parts
// stay normal, and the result is scaled back by 2^-28 (exact).  The fp16x2 mode
// splits only L: C = Lhi.Rhi + Llo.Rhi, R rounded once to float16 (relative
// error <= 2^-11 per R value, 1 - F ~ 1e-7): two MFMAs and two thirds of the
// operand loads of the three-product modes.
//
// Layout: L and R are stored in MFMA fragment order, so that each wavefront's
// operand load for one 32x32x16 step is one contiguous 1 KiB:
//   Lf[(rb * S + s) * 64 + lane][e] = L[32 rb + lane % 32][16 s + 8 (lane / 32) + e]
//   Rf[(cb * S + s) * 64 + lane][e] = R[16 s + 8 (lane / 32) + e][32 cb + lane % 32]
// with S = ceil(2K / 16) steps (the inner dimension is zero-padded).
//
// Tiles: a workgroup (4 wavefronts, 2 x 2) owns 128 rows x 256 real columns
// at a time; each wavefront 64 x 128 = 2 x 4 blocks of 32 x 32.  Consecutive
// workgroups land on consecutive XCDs; each XCD is given one band of columns
// so that the R fragments of its band stay in its L2 while rows stream
// through.  With a capped grid the kernel is persistent: workgroups loop over
// tiles, so a tile's stores drain while the next tile is computed.
#include "ccut_internal.h"
#include "merge_mfma.h"

#include <type_traits>

namespace ccut {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// 16-byte stores whose data registers the next vector instructions may overwrite.  The
// store reads its four data registers over several cycles after it issues, and the
// compiler does not keep a following vector write away from them: in a GEMM variant
// that wrote one instruction behind such a store, the last quarter of each 16-lane
// group stored the new value of the first register (wrong .x words in 16-amplitude
// pieces, different from run to run).  Nothing is scheduled in the few cycles after
// these stores.
__device__ __forceinline__ void store16_nt(f32x4 v, f32x4* p) {
  __builtin_nontemporal_store(v, p);
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_nop 4" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr bool is_f16(int mode) { return mode == MERGE_FP16X3 || mode == MERGE_FP16X2; }

template <int MODE>
__device__ __forceinline__ void split_value(float v, uint16_t& hi, uint16_t& lo) {
  if (is_f16(MODE)) {
    const float s = v * 16384.0f;  // 2^14
    const _Float16 h = (_Float16)s;
    const _Float16 l = (_Float16)(s - (float)h);
    hi = __builtin_bit_cast(uint16_t, h);
    lo = __builtin_bit_cast(uint16_t, l);
  } else {
    hi = bf16_rne(v);
    lo = bf16_rne(v - bf16_to_f(hi));
  }
}

// ------------------------------------------------------------ split kernel
__device__ __forceinline__ uint4 pack8(const uint16_t (&v)[8]) {
  uint4 r;
  r.x = v[0] | ((uint32_t)v[1] << 16); r.y = v[2] | ((uint32_t)v[3] << 16);
  r.z = v[4] | ((uint32_t)v[5] << 16); r.w = v[6] | ((uint32_t)v[7] << 16);
  return r;
}

// R fragment of thread t (one (cb, s, lane)) for batch entry beta.  The fp16x2
// mode never reads Rlo, so it is not written.
template <int MODE>
__device__ __forceinline__ void split_R_one(uint64_t t, int beta, const float2* __restrict__ A, uint64_t a_kstride,
                                            uint64_t a_bstride, const float2* __restrict__ w, int K, int S,
                                            uint4* __restrict__ hi, uint4* __restrict__ lo, uint64_t plane_stride) {
  const int lane = (int)(t & 63);
  const uint64_t cs = t >> 6;
  const int s = (int)(cs % S);
  const uint64_t cb = cs / S;
  const uint64_t c = cb * 32 + (lane & 31);
  const uint64_t x = c >> 1;
  const int part = (int)(c & 1);
  const float2* Ab = A + beta * a_bstride + x;
  uint16_t h[8], l[8];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int k = 8 * s + 4 * (lane >> 5) + p;  // kappa = 2k + comp
    float2 av = make_float2(0.f, 0.f);
    if (k < K) {
      const float2 a = Ab[(uint64_t)k * a_kstride];
      const float2 wk = w[k];
      av = make_float2(wk.x * a.x - wk.y * a.y, wk.x * a.y + wk.y * a.x);
    }
    const float r0 = part == 0 ? av.x : av.y;   // comp 0
    const float r1 = part == 0 ? -av.y : av.x;  // comp 1
    split_value<MODE>(r0, h[2 * p], l[2 * p]);
    split_value<MODE>(r1, h[2 * p + 1], l[2 * p + 1]);
  }
  hi[beta * plane_stride + t] = pack8(h);
  if (MODE != MERGE_FP16X2) lo[beta * plane_stride + t] = pack8(l);
}

// L fragment of thread t (one (rb, s, lane)) for batch entry beta.
template <int MODE>
__device__ __forceinline__ void split_L_one(uint64_t t, int beta, const float2* __restrict__ B, uint64_t b_kstride,
                                            uint64_t b_bstride, int K, int S, uint4* __restrict__ hi,
                                            uint4* __restrict__ lo, uint64_t plane_stride) {
  const int lane = (int)(t & 63);
  const uint64_t rs = t >> 6;
  const int s = (int)(rs % S);
  const uint64_t rb = rs / S;
  const uint64_t y = rb * 32 + (lane & 31);
  const float2* Bb = B + beta * b_bstride + y;
  uint16_t h[8], l[8];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int k = 8 * s + 4 * (lane >> 5) + p;
    const float2 b = k < K ? Bb[(uint64_t)k * b_kstride] : make_float2(0.f, 0.f);
    split_value<MODE>(b.x, h[2 * p], l[2 * p]);
    split_value<MODE>(b.y, h[2 * p + 1], l[2 * p + 1]);
  }
  hi[beta * plane_stride + t] = pack8(h);
  lo[beta * plane_stride + t] = pack8(l);
}

// Both operands in one launch: workgroups [0, r_blocks) write R fragments
// (batch entries < r_batch), the rest L fragments (batch entries < batch).
template <int MODE>
__global__ __launch_bounds__(256) void k_split(MergeMfmaArgs a, int r_blocks) {
  const int beta = blockIdx.y;
  if ((int)blockIdx.x < r_blocks) {
    if (beta >= a.r_batch) return;
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= ((uint64_t)1 << (a.qx + 1 - 5)) * a.S * 64) return;
    split_R_one<MODE>(t, beta, a.A, a.a_kstride, a.a_bstride, a.w, a.K, a.S, a.Rhi, a.Rlo, a.r_plane_stride);
  } else {
    if (beta >= a.batch) return;
    const uint64_t t = (uint64_t)(blockIdx.x - r_blocks) * 256 + threadIdx.x;
    if (t >= ((uint64_t)1 << (a.qy - 5)) * a.S * 64) return;
    split_L_one<MODE>(t, beta, a.B, a.b_kstride, a.b_bstride, a.K, a.S, a.Lhi, a.Llo, a.l_plane_stride);
  }
}

// ------------------------------------------------------------- GEMM kernel
template <int MODE>
__device__ __forceinline__ f32x16 mfma(uint4 a, uint4 b, f32x16 c) {
  if (is_f16(MODE)) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                  c, 0, 0, 0);
  }
}

// EPI 0: every lane stores its accumulators directly (4-byte non-temporal stores,
//        two full 128-byte rows per instruction).
// EPI 1: each wavefront writes a 32-row slab through LDS and stores it back as
//        16-byte chunks, two 512-byte row segments per instruction.
constexpr int EPI_LDS_ROW = 128 + 4;  // floats per LDS row (padded)

template <int MODE, int EPI, int RBW>
__global__ __launch_bounds__(256) void k_merge_gemm(const uint4* __restrict__ Lhi, const uint4* __restrict__ Llo,
                                                    const uint4* __restrict__ Rhi, const uint4* __restrict__ Rlo,
                                                    uint64_t l_bstride, uint64_t r_bstride, float* __restrict__ out,
                                                    uint64_t out_bstride, int qx, int qy, int S, int col_tiles,
                                                    int row_tiles) {
  // RBW: 32-row blocks per wavefront (2: 64 x 128 per wavefront, 128 x 256 per
  // workgroup; 1: 32 x 128 and 64 x 256, half the accumulators so that more
  // workgroups share a CU and one's stores drain while another computes).
  const int beta = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lstep = (uint64_t)S * 64;  // next 32-row (or column) block
  __shared__ __align__(16) float smem_f[EPI == 1 ? 4 * 16 * EPI_LDS_ROW : 4];
  constexpr bool L_SPLIT = MODE != MERGE_BF16;
  constexpr bool R_SPLIT = MODE == MERGE_BF16X3 || MODE == MERGE_FP16X3;
  const float scale = is_f16(MODE) ? (1.0f / 268435456.0f) : 1.0f;  // 2^-28
  const uint64_t ncols = (uint64_t)2 << qx;
  float* ob = out + beta * out_bstride;
  const int ntiles = col_tiles * row_tiles;
  // Tile loop (persistent when the grid is capped).  Workgroup b runs on XCD b % 8;
  // with whole XCD bands the workgroups of one XCD sweep the tiles of one column
  // band, so the band's R fragments stay in that XCD's L2.
  const bool banded = (col_tiles & 7) == 0 && (gridDim.x & 7) == 0;
  const int band = col_tiles >> 3;
  const int step = banded ? (int)(gridDim.x >> 3) : (int)gridDim.x;
  const int first = banded ? (int)(blockIdx.x >> 3) : (int)blockIdx.x;
  const int limit = banded ? ntiles >> 3 : ntiles;
  for (int i = first; i < limit; i += step) {
    int trow, tcol;
    if (banded) {
      trow = i / band;
      tcol = (int)(blockIdx.x & 7) * band + i % band;
    } else {
      trow = i / col_tiles;
      tcol = i % col_tiles;
    }
    const int rb0 = trow * (2 * RBW) + (wave >> 1) * RBW;  // 32-row blocks of this wave
    const int cb0 = tcol * 8 + (wave & 1) * 4;             // 32-column blocks of this wave
    const uint4* lh = Lhi + beta * l_bstride + ((uint64_t)rb0 * S) * 64 + lane;
    const uint4* ll = Llo + beta * l_bstride + ((uint64_t)rb0 * S) * 64 + lane;
    const uint4* rh = Rhi + beta * r_bstride + ((uint64_t)cb0 * S) * 64 + lane;
    const uint4* rl = Rlo + beta * r_bstride + ((uint64_t)cb0 * S) * 64 + lane;

    f32x16 acc[RBW][4];
#pragma unroll
    for (int r = 0; r < RBW; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[r][c][v] = 0.f;

    if constexpr (RBW == 2) {
      // 128-row tiles (128 accumulator registers: few wavefronts per SIMD, so each must
      // hide its own load latency): two operand buffers filled alternately, so the
      // loads of step s + 1 are in flight while the MFMAs of step s run; the scheduler
      // barriers keep the compiler from sinking them below those MFMAs, and no register
      // copies tie them to the current step.  Measured: q = 30, K = 256 merges
      // 6.4 -> 4.6 ms.  The 64-row tiles rely on four wavefronts per SIMD instead; the
      // second buffer would cost them that occupancy.
      struct Frag {
        uint4 a_hi[RBW], a_lo[RBW], b_hi[4], b_lo[4];
      };
      auto load = [&](Frag& f, int st) {
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
          f.a_hi[r] = lh[r * lstep + st * 64];
          if (L_SPLIT) f.a_lo[r] = ll[r * lstep + st * 64];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          f.b_hi[c] = rh[c * lstep + st * 64];
          if (R_SPLIT) f.b_lo[c] = rl[c * lstep + st * 64];
        }
      };
      auto mma = [&](const Frag& f) {
#pragma unroll
        for (int r = 0; r < RBW; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            if (L_SPLIT) acc[r][c] = mfma<MODE>(f.a_lo[r], f.b_hi[c], acc[r][c]);
            if (R_SPLIT) acc[r][c] = mfma<MODE>(f.a_hi[r], f.b_lo[c], acc[r][c]);
            acc[r][c] = mfma<MODE>(f.a_hi[r], f.b_hi[c], acc[r][c]);
          }
      };
      Frag fa, fb;
      load(fa, 0);
      int s = 0;
      for (; s + 1 < S; s += 2) {
        load(fb, s + 1);
        __builtin_amdgcn_sched_barrier(0);
        mma(fa);
        load(fa, s + 2 < S ? s + 2 : s + 1);  // past the end: reload step s + 1 (unused)
        __builtin_amdgcn_sched_barrier(0);
        mma(fb);
      }
      if (s < S) mma(fa);  // odd S: the last step
    } else {
      for (int s = 0; s < S; ++s) {
        uint4 a_hi[RBW], a_lo[RBW], b_hi[4], b_lo[4];
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
          a_hi[r] = lh[r * lstep + s * 64];
          if (L_SPLIT) a_lo[r] = ll[r * lstep + s * 64];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          b_hi[c] = rh[c * lstep + s * 64];
          if (R_SPLIT) b_lo[c] = rl[c * lstep + s * 64];
        }
#pragma unroll
        for (int r = 0; r < RBW; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            if (L_SPLIT) acc[r][c] = mfma<MODE>(a_lo[r], b_hi[c], acc[r][c]);
            if (R_SPLIT) acc[r][c] = mfma<MODE>(a_hi[r], b_lo[c], acc[r][c]);
            acc[r][c] = mfma<MODE>(a_hi[r], b_hi[c], acc[r][c]);
          }
      }
    }
    if (EPI == 0) {
#pragma unroll
      for (int r = 0; r < RBW; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint64_t col = (uint64_t)(cb0 + c) * 32 + (lane & 31);
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const uint64_t row = (uint64_t)(rb0 + r) * 32 + (v & 3) + 4 * (lane >> 5) + 8 * (v >> 2);
            __builtin_nontemporal_store(acc[r][c][v] * scale, ob + row * ncols + col);
          }
        }
    } else {
      // 16-row half slabs per wavefront: accumulator registers v < 8 hold rows 0..15
      float* my = smem_f + wave * 16 * EPI_LDS_ROW;
#pragma unroll
      for (int r = 0; r < RBW; ++r) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
          for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int v = 8 * h; v < 8 * h + 8; ++v) {
              const int row = (v & 3) + 4 * (lane >> 5) + 8 * ((v >> 2) & 1);
              my[row * EPI_LDS_ROW + c * 32 + (lane & 31)] = acc[r][c][v];
            }
          // the slab is this wavefront's own: its LDS ops execute in order, so a
          // wavefront-scope fence (no workgroup barrier) orders the writes and reads
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          // lanes 0..31 cover one 128-float row, lanes 32..63 the next
          const uint64_t col0 = (uint64_t)cb0 * 32 + 4 * (lane & 31);
#pragma unroll
          for (int rr = 0; rr < 16; rr += 2) {
            const int row = rr + (lane >> 5);
            f32x4 v = *reinterpret_cast<const f32x4*>(my + row * EPI_LDS_ROW + 4 * (lane & 31));
            v *= scale;
            const uint64_t grow = (uint64_t)(rb0 + r) * 32 + 16 * h + row;
            store16_nt(v, reinterpret_cast<f32x4*>(ob + grow * ncols + col0));
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
        }
      }
    }
  }
  (void)qy;
}

// ------------------------------------------- R-stationary GEMM (K <= 64)
// One workgroup of 16 wavefronts per CU owns a strip of 256 real columns (8
// column blocks) and keeps the strip's R fragments for every step (hi and lo;
// at most 8 steps: 128 KiB) in LDS for its whole life.  Each wavefront sweeps
// its own 32-row blocks (w, w + 16, ...) independently: it holds the block's L
// fragments for all steps in registers and runs the strip in four passes of two
// column blocks, reading R from LDS.  L2 serves half the output size in operand
// bytes (the tiled kernel above: 3x to 5x).
// Stores and loads share one in-order counter, so a wavefront that loads after
// storing waits for its stores to drain.  The next block's L fragments are
// therefore fetched during the last pass (into the registers of the steps that
// pass has already used) before that pass's stores, and the first block is peeled
// so that every path into the loop has the same load/store order (the compiler
// then waits only for the loads, not for the stores issued after them).
// Stores are buffer stores: a wave-uniform base, one lane offset and the row
// offset in a scalar, each access range-checked by the hardware.
constexpr int RS_WAVES = 16;
constexpr int RS_NC = 8;  // column blocks per strip

template <int MODE, int S>
__global__ __launch_bounds__(RS_WAVES * 64) void k_merge_gemm_rs(
    const uint4* __restrict__ Lhi, const uint4* __restrict__ Llo, const uint4* __restrict__ Rhi,
    const uint4* __restrict__ Rlo, uint64_t l_bstride, uint64_t r_bstride, float* __restrict__ out,
    uint64_t out_bstride, int qx, int qy, int strips, int row_split) {
  constexpr bool L_SPLIT = MODE != MERGE_BF16;
  constexpr bool R_SPLIT = MODE == MERGE_BF16X3 || MODE == MERGE_FP16X3;
  constexpr int CB = 2;  // column blocks per pass
  // R fragments in LDS: index ((cb * S + s) * NP + plane) * 64 + lane, hi and lo of one
  // (column block, step) side by side so that a pass's reads sit within the 64 KiB
  // reach of one base address plus immediate offsets
  constexpr int NP = R_SPLIT ? 2 : 1;
  __shared__ uint4 sR[RS_NC * S * NP * 64];
  const int beta = blockIdx.y;
  const int strip = (int)blockIdx.x % strips;
  const int part = (int)blockIdx.x / strips;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const float scale = is_f16(MODE) ? (1.0f / 268435456.0f) : 1.0f;  // 2^-28
  const uint32_t ncols = 2u << qx;
  float* ob = out + beta * out_bstride;
  const char* out_end = reinterpret_cast<const char*>(ob + ((uint64_t)1 << qy) * ncols);

  {  // the strip's R fragments: 8 column blocks x S steps, contiguous in both planes
    constexpr int n = RS_NC * S * 64;
    const uint4* gh = Rhi + beta * r_bstride + (uint64_t)strip * n;
    const uint4* gl = Rlo + beta * r_bstride + (uint64_t)strip * n;
    for (int i = threadIdx.x; i < n; i += RS_WAVES * 64) {
      const int d = (i >> 6) * NP * 64 + (i & 63);
      sR[d] = gh[i];
      if (R_SPLIT) sR[d + 64] = gl[i];
    }
  }
  __syncthreads();

  const int nrb = 1 << (qy - 5);
  const int per = (nrb + row_split - 1) / row_split;
  const int rb_begin = part * per;
  const int rb_end = min(nrb, rb_begin + per);
  const uint4* lbh = Lhi + beta * l_bstride;
  const uint4* lbl = Llo + beta * l_bstride;
  // byte offset of this lane's first accumulator within a 32-row block
  const uint32_t o_st = ((uint32_t)(4 * (lane >> 5)) * ncols + (uint32_t)(lane & 31)) * 4u;
  uint4 Lh[S], Ll[S];
  // L fragments of steps [s0, s0 + n) of row block r (always in bounds: r < nrb)
  auto loadL = [&](int r, int s0, int n) {
    const char* bh = reinterpret_cast<const char*>(lbh + (uint64_t)r * S * 64);
    const char* bl = reinterpret_cast<const char*>(lbl + (uint64_t)r * S * 64);
    const uint32_t lo16 = (uint32_t)lane * 16u;
#pragma unroll
    for (int t = 0; t < S; ++t)
      if (t >= s0 && t < s0 + n) {
        Lh[t] = *reinterpret_cast<const uint4*>(bh + (lo16 + t * 1024u));
        if (L_SPLIT) Ll[t] = *reinterpret_cast<const uint4*>(bl + (lo16 + t * 1024u));
      }
  };
  auto block = [&](int rb) {
    const int nx = min(rb + RS_WAVES, nrb - 1);  // past the last block: a valid block, never used
    float* orow = ob + (uint64_t)rb * 32 * ncols + (uint64_t)strip * (RS_NC * 32);
#pragma unroll
    for (int p = 0; p < RS_NC / CB; ++p) {
      constexpr int kLast = RS_NC / CB - 1;
      f32x16 acc[CB];
#pragma unroll
      for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[c][v] = 0.f;
      const uint4* rp = sR + (CB * p) * S * NP * 64 + lane;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        uint4 bh[CB], bl[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          bh[c] = rp[(c * S + s) * NP * 64];
          if (R_SPLIT) bl[c] = rp[(c * S + s) * NP * 64 + 64];
        }
        if (L_SPLIT) {
#pragma unroll
          for (int c = 0; c < CB; ++c) acc[c] = mfma<MODE>(Ll[s], bh[c], acc[c]);
        }
        if (R_SPLIT) {
#pragma unroll
          for (int c = 0; c < CB; ++c) acc[c] = mfma<MODE>(Lh[s], bl[c], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[c] = mfma<MODE>(Lh[s], bh[c], acc[c]);
        if (p == kLast) {
          // registers of steps this pass is done with take the next block's fragments
          if (S == 1) {
            __builtin_amdgcn_sched_barrier(0);
            loadL(nx, 0, 1);
            __builtin_amdgcn_sched_barrier(0);
          } else if (s == S / 2 - 1 || s == S - 1) {
            __builtin_amdgcn_sched_barrier(0);
            loadL(nx, s == S - 1 ? S / 2 : 0, S / 2);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        if (is_f16(MODE)) acc[c] *= scale;
        float* oc = orow + (CB * p + c) * 32;
        const uint64_t left = (uint64_t)(out_end - reinterpret_cast<const char*>(oc));
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            oc, 0, (int)(left > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)left), 0x00020000);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const uint32_t soff = (uint32_t)((v & 3) + 8 * (v >> 2)) * ncols * 4u;
          // non-temporal (cache policy bit 1)
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc[c][v]), rs, (int)o_st, (int)soff, 2);
        }
      }
    }
  };
  int rb = rb_begin + wave;
  loadL(min(rb, nrb - 1), 0, S);
  if (rb < rb_end) {
    block(rb);
    for (rb += RS_WAVES; rb < rb_end; rb += RS_WAVES) block(rb);
  }
}

// 16-byte items as a native vector type: HIP's uint4 is copied through memcpy,
// which keeps arrays of it out of registers
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;

// ------------------------------------------ LDS-staged GEMM (large K)
// For many MFMA steps the tiled kernel above loads every wavefront's fragments
// from L2 on their own (3 to 5 times the output size in all).  Here a workgroup
// of 8 wavefronts (4 x 2) owns a 256-row x 256-column tile, each wavefront
// 64 x 128 (2 x 4 blocks of 32 x 32): per MFMA step the tile's 8 L and 8 R
// fragments (both planes: 32 KiB in the three-product modes) are copied from L2
// straight into LDS once, four steps ahead, into one of four buffers; every
// wavefront reads its own fragments of the next step into a second register set
// before it issues the MFMAs of the current one.  Per step and output block the
// products run in the tiled kernel's order (lo.hi, hi.lo, hi.hi), so the results
// are the same bit for bit.  One workgroup per CU, persistent over the tiles; the
// stream of steps runs on across tiles, so a tile's stores (through LDS, 4-row
// slabs, 512-byte row segments) go out behind the next tile's first copies.
// Measured at q = 30, K = 256 against the tiled kernel: fp16x3 5.0 to 5.9 ms
// against 7.4 ms, fp16x2 3.7 to 4.0 against 4.8 ms, unsplit bf16 2.4 against
// 3.9 ms.  The shader clock drops to 1.35 to 1.6 GHz under this load; in cycles
// the fp16x3 kernel takes 7.38 M, of which its MFMAs need 6.29 M and the tile
// stores (256 KiB per CU and tile through the vector memory path) most of the rest.
constexpr int LK_WAVES = 8;

// global stores of one wavefront's share of a tile: 2 block rows x 8 slabs x 2 row pairs
constexpr int LK_EPI_STORES = 32;

// Waits until at most N vector memory operations of this wavefront are outstanding
// and all its LDS operations are done, then the workgroup barrier.  Written out
// because the barrier builtin's fence would wait for every outstanding copy into LDS;
// the wait is the compiler's own instruction, so its later waits know of it (gfx9
// fields: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
template <int N>
__device__ __forceinline__ void lk_wait_barrier() {
  static_assert(N >= 0 && N < 64, "vmcnt field");
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// 16 bytes per lane from global memory straight into LDS: lane i's bytes land at
// dst + 16 i (dst uniform over the wavefront); counted by the vector memory counter
__device__ __forceinline__ void lds_copy16(const u32x4* src, u32x4* dst) {
  __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
}

template <int PER>
struct LkSrc {  // per copy of a wavefront: its fragment's block base, L or R
  const u32x4* src[PER];
  bool is_l[PER];
};

template <int MODE>
__global__ __launch_bounds__(LK_WAVES * 64) void k_merge_gemm_lk(
    const uint4* __restrict__ Lhi, const uint4* __restrict__ Llo, const uint4* __restrict__ Rhi,
    const uint4* __restrict__ Rlo, uint64_t l_bstride, uint64_t r_bstride, float* __restrict__ out,
    uint64_t out_bstride, int qx, int S, int col_tiles, int row_tiles) {
  constexpr bool L_SPLIT = MODE != MERGE_BF16;
  constexpr bool R_SPLIT = MODE == MERGE_BF16X3 || MODE == MERGE_FP16X3;
  constexpr int LP = L_SPLIT ? 2 : 1, RP = R_SPLIT ? 2 : 1;
  constexpr int NF = 8 * LP + 8 * RP;             // fragments per step: L (block, plane), then R
  constexpr int PER = NF * 64 / (LK_WAVES * 64);  // 16-byte items each thread copies per step
  constexpr int BUF = NF * 64;                    // items per LDS buffer
  constexpr int SLAB = 4 * EPI_LDS_ROW;           // floats of one wavefront's epilogue slab
  // operand buffers of steps g = 0, 1, 2, 3 mod 4: four arrays, each touched at fixed
  // places of the unrolled loop, so that the compiler can tell a step's reads from the
  // copies still landing in the other buffers
  __shared__ u32x4 ops0[BUF], ops1[BUF], ops2[BUF], ops3[BUF];
  __shared__ float slabs[LK_WAVES * SLAB];  // epilogue, apart from the operand buffers
  const int beta = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;  // 2 row blocks and 4 column blocks each
  const float scale = is_f16(MODE) ? (1.0f / 268435456.0f) : 1.0f;  // 2^-28
  const uint64_t ncols = (uint64_t)2 << qx;
  float* ob = out + beta * out_bstride;
  const uint64_t lstep = (uint64_t)S * 64;
  const u32x4* lbh = reinterpret_cast<const u32x4*>(Lhi + beta * l_bstride);
  const u32x4* lbl = reinterpret_cast<const u32x4*>(Llo + beta * l_bstride);
  const u32x4* rbh = reinterpret_cast<const u32x4*>(Rhi + beta * r_bstride);
  const u32x4* rbl = reinterpret_cast<const u32x4*>(Rlo + beta * r_bstride);

  // Tiles of this workgroup.  Workgroup b runs on XCD b % 8.  Grouped order (a grid
  // of 8 x 32 workgroups): XCD x owns the column band of tiles [x band, (x + 1) band)
  // and its 32 workgroups take 4 x 8 tiles of it at a time, rounds sweeping the
  // band's 8-tile column groups, then its 4-tile row groups, so that L2 serves each
  // row tile's fragments to 8 workgroups and each column tile's to 4.  Otherwise,
  // banded or plain order as in the tiled kernel.
  const int ntiles = col_tiles * row_tiles;
  const int per_xcd = (int)(gridDim.x >> 3);
  const bool grouped = (gridDim.x & 7) == 0 && per_xcd == 32 && col_tiles % 64 == 0 && row_tiles % 4 == 0;
  const bool banded = !grouped && (col_tiles & 7) == 0 && (gridDim.x & 7) == 0;
  const int band = col_tiles >> 3;
  const int w = (int)(blockIdx.x >> 3), xcd = (int)(blockIdx.x & 7);
  int mine;
  if (grouped) {
    mine = ntiles / (int)gridDim.x;  // every round gives each workgroup one tile
  } else {
    const int tstep = banded ? per_xcd : (int)gridDim.x;
    const int first = banded ? w : (int)blockIdx.x;
    const int limit = banded ? ntiles >> 3 : ntiles;
    mine = (limit - first + tstep - 1) / tstep;  // >= 1: the grid never exceeds the tiles
  }
  const int steps = mine * S;
  const int cgroups = band / 8;  // grouped: 8-tile column groups per band
  // t-th tile of this workgroup (selects, no branches: the loads must stay in one basic
  // block with the MFMAs they overlap, or the compiler sinks them to their use)
  auto tile_rc = [&](int t, int& tr, int& tc) {
    const int tstep = banded ? per_xcd : (int)gridDim.x;
    const int i = (banded ? w : (int)blockIdx.x) + t * tstep;
    const int div = banded ? band : col_tiles;
    const int gr = t / cgroups, gc = t % cgroups;
    tr = grouped ? gr * 4 + (w >> 3) : i / div;
    tc = grouped ? xcd * band + gc * 8 + (w & 7) : (banded ? xcd * band : 0) + i % div;
  };

  // this wavefront's share of a step's fragments: its copy j carries fragment
  // f = 8 j + wave (f < 8 LP: L block f / LP, plane f % LP; then R block (f - 8 LP) / RP,
  // plane (f - 8 LP) % RP), lane l its 16 bytes l; the block's base is uniform over the
  // wavefront, only tile and step move
  LkSrc<PER> q;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int f = j * LK_WAVES + wave;
    q.is_l[j] = f < 8 * LP;
    const int blk = q.is_l[j] ? f / LP : (f - 8 * LP) / RP;
    const int pl = q.is_l[j] ? f % LP : (f - 8 * LP) % RP;
    q.src[j] = (q.is_l[j] ? (pl ? lbl : lbh) : (pl ? rbl : rbh)) + (uint64_t)blk * lstep;
  }
  // Copy stream: a round's four copies are steps dk .. dk + 3 of this workgroup's tile
  // dt (S is a multiple of 4, so a round never crosses tiles; past the last tile, the
  // last again: in bounds, never read).  Each wavefront's 64 items of a copy land in
  // LDS as 1 KiB, lane after lane.  The tile's bases change once per S steps.
  uint64_t c_lo = 0, c_ro = 0;
  int dt = 0, dk = 0;
  auto copy_tile = [&]() {
    int tr, tc;
    tile_rc(dt < mine ? dt : mine - 1, tr, tc);
    c_lo = (uint64_t)tr * 8 * lstep;
    c_ro = (uint64_t)tc * 8 * lstep;
  };
  auto dma = [&](u32x4* buf, int j4) {
    const uint64_t so = (uint64_t)(dk + j4) * 64;
    u32x4* d = buf + wave * 64;
#pragma unroll
    for (int j = 0; j < PER; ++j) lds_copy16(q.src[j] + (q.is_l[j] ? c_lo : c_ro) + so + lane, d + j * LK_WAVES * 64);
  };
  auto next_round = [&]() {
    dk += 4;
    if (dk == S) {
      dk = 0;
      ++dt;
      copy_tile();
    }
  };

  f32x16 acc[2][4];
  struct Frags {
    uint4 a_hi[2], a_lo[2], b_hi[4], b_lo[4];
  };
  // a step's fragments of this wavefront, from LDS
  auto read = [&](Frags& f, const u32x4* buf) {
    const u32x4* b = buf + lane;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      f.a_hi[r] = __builtin_bit_cast(uint4, b[((wr * 2 + r) * LP) * 64]);
      if (L_SPLIT) f.a_lo[r] = __builtin_bit_cast(uint4, b[((wr * 2 + r) * LP + 1) * 64]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      f.b_hi[c] = __builtin_bit_cast(uint4, b[(8 * LP + (wc * 4 + c) * RP) * 64]);
      if (R_SPLIT) f.b_lo[c] = __builtin_bit_cast(uint4, b[(8 * LP + (wc * 4 + c) * RP + 1) * 64]);
    }
  };
  // a step's MFMAs in the tiled kernel's order
  auto compute = [&](const Frags& f) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (L_SPLIT) acc[r][c] = mfma<MODE>(f.a_lo[r], f.b_hi[c], acc[r][c]);
        if (R_SPLIT) acc[r][c] = mfma<MODE>(f.a_hi[r], f.b_lo[c], acc[r][c]);
        acc[r][c] = mfma<MODE>(f.a_hi[r], f.b_hi[c], acc[r][c]);
      }
  };
  // 4-row slabs per wavefront through LDS, 512-byte row segments
  auto epilogue = [&](int t) {
    int tr, tc;
    tile_rc(t, tr, tc);
    float* my = slabs + wave * SLAB;
    const int rb0 = tr * 8 + wr * 2, cb0 = tc * 8 + wc * 4;
    const uint64_t col0 = (uint64_t)cb0 * 32 + 4 * (lane & 31);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
      for (int h = 0; h < 8; ++h) {  // accumulator registers 2 h, 2 h + 1: block rows
                                     // 8 (h / 2) + 4 (lane / 32) + 2 (h % 2) + (v & 1)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int v = 2 * h; v < 2 * h + 2; ++v)
            my[((v & 1) + 2 * (lane >> 5)) * EPI_LDS_ROW + c * 32 + (lane & 31)] = acc[r][c][v];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int rr = 0; rr < 4; rr += 2) {
          const int row = rr + (lane >> 5);  // slab row: (v & 1) + 2 (writer's lane / 32)
          f32x4 v = *reinterpret_cast<const f32x4*>(my + row * EPI_LDS_ROW + 4 * (lane & 31));
          v *= scale;
          const int brow = 8 * (h >> 1) + 4 * (row >> 1) + 2 * (h & 1) + (row & 1);
          const uint64_t grow = (uint64_t)(rb0 + r) * 32 + brow;
          store16_nt(v, reinterpret_cast<f32x4*>(ob + grow * ncols + col0));
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
    }
  };
  auto clear = [&]() {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[r][c][v] = 0.f;
  };

  // Entering step g: its fragments are in registers (or on their way from LDS), LDS
  // holds step g + 1, and steps g + 2 and g + 3 are on their way into LDS.  Step g
  // reads step g + 1's fragments into the other register set, loads step g + 4 into the
  // buffer step g left (all its reads ended before the last barrier), issues its MFMAs,
  // and waits for its own copies of step g + 2 before the barrier that makes them
  // visible to all.  S is a multiple of 4, so tiles end in the fourth step of a round;
  // the memory counter runs in order, so the first step after a tile's stores waits for
  // most of them as well.
  Frags f0, f1;
  copy_tile();
  dma(ops0, 0);
  dma(ops1, 1);
  lk_wait_barrier<PER>();  // step 0 in LDS
  read(f0, ops0);
  dma(ops2, 2);
  dma(ops3, 3);
  next_round();
  lk_wait_barrier<2 * PER>();  // step 1 in LDS, step 0 read by all
  clear();
  constexpr int NRD = 2 * LP + 4 * RP;  // LDS reads of a step's fragments
  constexpr int NMF = 8 * (LP + RP - 1);  // MFMAs of a step
  using Plain = std::integral_constant<bool, false>;
  using AfterStores = std::integral_constant<bool, true>;
  auto step = [&](Frags& cur, Frags& nxt, const u32x4* rd, u32x4* wr_buf, int j4, auto after_stores) {
    read(nxt, rd);
    dma(wr_buf, j4);  // step g + 4
    compute(cur);
    // issue order: the first MFMAs right after the barrier, the reads and copies in
    // between the MFMAs, so that the MFMA pipe does not wait for their issue
#pragma unroll
    for (int i = 0; i < NRD / 2; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
      __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);  // LDS reads
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
      __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // copy into LDS
    }
    __builtin_amdgcn_sched_group_barrier(0x008, NMF - NRD / 2 - PER, 0);
    if constexpr (decltype(after_stores)::value)
      lk_wait_barrier<2 * PER + LK_EPI_STORES>();  // the tile's stores may stay in flight
    else
      lk_wait_barrier<2 * PER>();
  };
  // a round of four steps; in the first round after a tile's stores the first two steps
  // wait only for the copies older than the stores (the third waits for them as well)
  auto round = [&](auto after_stores) {
    step(f0, f1, ops1, ops0, 0, after_stores);
    step(f1, f0, ops2, ops1, 1, after_stores);
    step(f0, f1, ops3, ops2, 2, Plain{});
    step(f1, f0, ops0, ops3, 3, Plain{});
    next_round();
  };
  // tile by tile, the first apart (no stores before it): each code path keeps the same
  // number of operations in flight, so the compiler's own waits stay exact
  const int rounds = S / 4;
  for (int r = 0; r < rounds; ++r) round(Plain{});
  epilogue(0);
  clear();
  for (int t = 1; t < mine; ++t) {
    round(AfterStores{});
    for (int r = 1; r < rounds; ++r) round(Plain{});
    epilogue(t);
    clear();
  }
  // the copies past the last step are still landing in LDS: not past the workgroup's end
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// ------------------------------- column-stationary GEMM with row-tile stores (K <= 64)
// The R-stationary kernel above runs at the speed of its store pattern: each store
// instruction writes two 128-byte row pieces, and its 16 wavefronts write 16
// different row blocks (stores alone in that pattern: 5.0 TB/s).  Here a workgroup
// of 8 wavefronts owns a 256-column strip and sweeps a range of 32-row blocks, one
// per round, with the work split by wavefront:
//  - wavefronts 0..3 compute: wavefront c keeps column blocks 2 c and 2 c + 1's R
//    fragments for every step in registers (hi and lo: at most 128 registers), reads
//    the round's L fragments from LDS one step ahead of the products, and writes its
//    two 32 x 32 results into an LDS tile of 32 rows x 256 columns;
//  - wavefronts 4..7 move data: each round they fetch the row block two rounds ahead
//    into registers, store the previous round's tile (8 rows of 1 KiB per wavefront,
//    16 bytes per lane: one whole row segment per instruction; stores alone in this
//    pattern reach 6.7 TB/s), then put the fetched fragments into LDS (a wait that
//    passes the stores just issued: the counter is in order and the loads came
//    first).
// L is triple-buffered and the tile double-buffered (115 KiB of LDS, one workgroup
// per CU), so one barrier per round orders everything.  The products are computed
// transposed (R fragments as the A operand, L as B), so that a lane holds four
// adjacent columns of one output row per register group and writes the tile 16 bytes
// at a time; per step they run in the tiled kernel's order (lo.hi, hi.lo, hi.hi), so
// the results are the same bit for bit.  Measured at q = 28, K = 64 in the pipeline
// (after a simulation, candidates alternated on one box): fp16x3 0.385 to 0.398 ms,
// bf16x3 0.366 to 0.372 ms, fp16x2 0.305 to 0.317 ms, against 0.400 to 0.406, 0.407
// to 0.413 and 0.411 to 0.423 ms for the R-stationary kernel.
constexpr int RC_PITCH = 260;  // floats per row of the LDS tile (256 + 4)

template <int MODE, int S>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void k_merge_gemm_rc(
    const uint4* __restrict__ Lhi, const uint4* __restrict__ Llo, const uint4* __restrict__ Rhi,
    const uint4* __restrict__ Rlo, uint64_t l_bstride, uint64_t r_bstride, float* __restrict__ out,
    uint64_t out_bstride, int qx, int qy, int strips, int row_split) {
  constexpr bool L_SPLIT = MODE != MERGE_BF16;
  constexpr bool R_SPLIT = MODE == MERGE_BF16X3 || MODE == MERGE_FP16X3;
  constexpr int LP = L_SPLIT ? 2 : 1;
  constexpr int ND = 256;                        // data threads
  constexpr int NL = S * LP * 64;                // 16-byte L items of one row block
  constexpr int LPT = NL >= ND ? NL / ND : 1;    // items each data thread fetches
  static_assert(NL >= ND ? NL % ND == 0 : ND % NL == 0, "L items per thread");
  __shared__ u32x4 sL[3][NL];
  __shared__ float tile[2][32 * RC_PITCH];
  const int beta = blockIdx.y;
  const int strip = (int)blockIdx.x % strips;
  const int part = (int)blockIdx.x / strips;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool data = wave >= 4;
  const float scale = is_f16(MODE) ? (1.0f / 268435456.0f) : 1.0f;  // 2^-28
  const uint32_t ncols = 2u << qx;
  const int nrb = 1 << (qy - 5);
  const int per = (nrb + row_split - 1) / row_split;
  const int rb_begin = part * per;
  const int rb_end = min(nrb, rb_begin + per);
  if (rb_begin >= rb_end) return;  // the whole workgroup
  const int nr = rb_end - rb_begin;
  float* ob = out + beta * out_bstride + (uint64_t)strip * 256;
  const uint4* lbh = Lhi + beta * l_bstride;
  const uint4* lbl = Llo + beta * l_bstride;
  const int dt = tid - 256;  // data thread index (data wavefronts)

  // compute wavefront c: column blocks 2 c and 2 c + 1 of the strip
  uint4 Rh[2][S], Rl[2][S];
  if (!data) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const uint64_t o = ((uint64_t)(strip * 8 + 2 * wave + b) * S) * 64 + lane;
      const uint4* gh = Rhi + beta * r_bstride + o;
      const uint4* gl = Rlo + beta * r_bstride + o;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        Rh[b][s] = gh[s * 64];
        if (R_SPLIT) Rl[b][s] = gl[s * 64];
      }
    }
  }
  u32x4 lreg[LPT];
  auto fetch_l = [&](int rb) {
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
      const int i = (dt + j * ND) % NL;
      const int sp = i >> 6, s = sp / LP, plane = sp % LP;
      const uint4* src = (plane ? lbl : lbh) + ((uint64_t)rb * S + s) * 64 + (i & 63);
      lreg[j] = __builtin_bit_cast(u32x4, *src);
    }
  };
  auto put_l = [&](int buf) {
#pragma unroll
    for (int j = 0; j < LPT; ++j)
      if (NL >= ND || dt < NL) sL[buf][dt + j * ND] = lreg[j];
  };
  // data wavefront d stores rows d + 4 j of the tile, one 1 KiB row per instruction
  auto store_tile = [&](int rb, int buf) {
    float* orow = ob + (uint64_t)rb * 32 * ncols;
    const int d = wave - 4;
    f32x4 v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = *reinterpret_cast<const f32x4*>(&tile[buf][(d + 4 * j) * RC_PITCH + 4 * lane]);
#pragma unroll
    for (int j = 0; j < 8; ++j) store16_nt(v[j], reinterpret_cast<f32x4*>(orow + (uint64_t)(d + 4 * j) * ncols) + lane);
  };
  auto compute = [&](int n) {
    f32x16 acc[2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[b][v] = 0.f;
    const u32x4* lb = sL[n % 3] + lane;
    u32x4 cur[LP], nxt[LP];
#pragma unroll
    for (int p = 0; p < LP; ++p) cur[p] = lb[p * 64];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (s + 1 < S) {
#pragma unroll
        for (int p = 0; p < LP; ++p) nxt[p] = lb[((s + 1) * LP + p) * 64];
      }
      __builtin_amdgcn_sched_barrier(0);
      const uint4 lh = __builtin_bit_cast(uint4, cur[0]);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (L_SPLIT) acc[b] = mfma<MODE>(Rh[b][s], __builtin_bit_cast(uint4, cur[LP - 1]), acc[b]);
        if (R_SPLIT) acc[b] = mfma<MODE>(Rl[b][s], lh, acc[b]);
        acc[b] = mfma<MODE>(Rh[b][s], lh, acc[b]);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int p = 0; p < LP; ++p) cur[p] = nxt[p];
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if (is_f16(MODE)) acc[b] *= scale;
      float* t = &tile[n & 1][(lane & 31) * RC_PITCH + (2 * wave + b) * 32 + 4 * (lane >> 5)];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const f32x4 q = {acc[b][4 * j], acc[b][4 * j + 1], acc[b][4 * j + 2], acc[b][4 * j + 3]};
        *reinterpret_cast<f32x4*>(t + 8 * j) = q;
      }
    }
  };
  auto round = [&](int n, auto first) {
    if (data) {
      // the fetch goes out before the stores, so that waiting for it passes them
      fetch_l(rb_begin + min(n + 2, nr - 1));
      if (!decltype(first)::value) store_tile(rb_begin + n - 1, (n - 1) & 1);
      put_l((n + 2) % 3);
    } else {
      compute(n);
    }
    __syncthreads();
  };

  if (data) {
    fetch_l(rb_begin);
    put_l(0);
    fetch_l(rb_begin + min(1, nr - 1));
    put_l(1);
  }
  __syncthreads();
  round(0, std::true_type{});
  for (int n = 1; n < nr; ++n) round(n, std::false_type{});
  if (data) store_tile(rb_end - 1, (nr - 1) & 1);
}

// S in {1, 2, 4, 8} (K <= 64; K is a power of two) and row offsets of a 32-row block
// within 32 bits (the buffer stores' scalar offset): 2^(qx + 1) floats per row, qx <= 23
bool merge_rs_supported(int qx, int S) { return qx >= 7 && qx <= 23 && (S == 1 || S == 2 || S == 4 || S == 8); }

// 256 x 256 tiles: at least one tile each way; MFMA steps a multiple of 4 (K >= 32)
bool merge_lk_supported(int qx, int qy, int S) { return qx >= 7 && qy >= 8 && S % 4 == 0; }

int cu_count() {
  int dev = 0, c = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0)
    return c;
  return 256;
}

template <int MODE>
int launch_mode(const MergeMfmaArgs& a, int variant, int grid_cap, hipStream_t s) {
  const int S = a.S;
  // split R (the A side, weights folded in; per batch entry unless shared) and L
  {
    const uint64_t nr = ((uint64_t)1 << (a.qx + 1 - 5)) * S * 64;
    const uint64_t nl = ((uint64_t)1 << (a.qy - 5)) * S * 64;
    const uint64_t r_blocks = (nr + 255) / 256, l_blocks = (nl + 255) / 256;
    if (r_blocks + l_blocks > 0x7FFFFFFFull) return fail(CCUT_EUNSUPPORTED, "merge operands too large to split");
    dim3 grid((unsigned)(r_blocks + l_blocks), std::max(a.batch, a.r_batch));
    ProfScope prof(PROF_SPLIT, s);
    hipLaunchKernelGGL(k_split<MODE>, grid, dim3(256), 0, s, a, (int)r_blocks);
    CCUT_HIP(hipGetLastError());
  }
  if (variant == 4 && merge_rs_supported(a.qx, S)) {
    // R-stationary kernel: one workgroup per (strip, row part, batch entry); row parts
    // only as many as it takes to give every CU one workgroup
    const int strips = 1 << (a.qx + 1 - 8);
    const int nrb = 1 << (a.qy - 5);
    const int want = (cu_count() + strips * a.batch - 1) / (strips * a.batch);
    const int row_split = std::max(1, std::min(want, nrb / RS_WAVES));
    if ((uint64_t)strips * row_split > 0x7FFFFFFFull) return fail(CCUT_EUNSUPPORTED, "merge too large");
    dim3 grid((unsigned)(strips * row_split), a.batch);
    const uint64_t r_bstride = a.r_batch > 1 ? a.r_plane_stride : 0;
    ProfScope prof(PROF_MERGE_GEMM, s);
#define CCUT_RS(SS)                                                                                              \
  hipLaunchKernelGGL((k_merge_gemm_rs<MODE, SS>), grid, dim3(RS_WAVES * 64), 0, s, a.Lhi, a.Llo, a.Rhi, a.Rlo,    \
                     a.l_plane_stride, r_bstride, a.out, a.out_bstride * 2, a.qx, a.qy, strips, row_split)
    switch (S) {
      case 1: CCUT_RS(1); break;
      case 2: CCUT_RS(2); break;
      case 4: CCUT_RS(4); break;
      default: CCUT_RS(8); break;
    }
#undef CCUT_RS
    CCUT_HIP(hipGetLastError());
    return 0;
  }
  if (variant == 6 && merge_rs_supported(a.qx, S)) {
    // column-stationary kernel: one workgroup per (strip, row part, batch entry), row
    // parts as many as it takes to give every CU one workgroup
    const int strips = 1 << (a.qx + 1 - 8);
    const int nrb = 1 << (a.qy - 5);
    const int want = (cu_count() + strips * a.batch - 1) / (strips * a.batch);
    const int row_split = std::max(1, std::min(want, nrb));
    if ((uint64_t)strips * row_split > 0x7FFFFFFFull) return fail(CCUT_EUNSUPPORTED, "merge too large");
    dim3 grid((unsigned)(strips * row_split), a.batch);
    const uint64_t r_bstride = a.r_batch > 1 ? a.r_plane_stride : 0;
    ProfScope prof(PROF_MERGE_GEMM, s);
#define CCUT_RC(SS)                                                                                              \
  hipLaunchKernelGGL((k_merge_gemm_rc<MODE, SS>), grid, dim3(512), 0, s, a.Lhi, a.Llo, a.Rhi, a.Rlo,              \
                     a.l_plane_stride, r_bstride, a.out, a.out_bstride * 2, a.qx, a.qy, strips, row_split)
    switch (S) {
      case 1: CCUT_RC(1); break;
      case 2: CCUT_RC(2); break;
      case 4: CCUT_RC(4); break;
      default: CCUT_RC(8); break;
    }
#undef CCUT_RC
    CCUT_HIP(hipGetLastError());
    return 0;
  }
  if (variant == 5 && merge_lk_supported(a.qx, a.qy, S)) {
    const int col_tiles = 1 << (a.qx + 1 - 8);
    const int row_tiles = 1 << (a.qy - 8);
    const int ntiles = col_tiles * row_tiles;
    // one workgroup per CU over all batch entries, a multiple of the 8 XCDs
    int per = std::max(1, cu_count() / std::max(1, a.batch));
    if (per >= 8) per &= ~7;
    dim3 grid((unsigned)std::min(ntiles, per), a.batch);
    const uint64_t r_bstride = a.r_batch > 1 ? a.r_plane_stride : 0;
    ProfScope prof(PROF_MERGE_GEMM, s);
    hipLaunchKernelGGL((k_merge_gemm_lk<MODE>), grid, dim3(LK_WAVES * 64), 0, s, a.Lhi, a.Llo, a.Rhi, a.Rlo,
                       a.l_plane_stride, r_bstride, a.out, a.out_bstride * 2, a.qx, S, col_tiles, row_tiles);
    CCUT_HIP(hipGetLastError());
    return 0;
  }
  if (variant >= 4) variant = 1;  // shapes the R-stationary or LDS-staged kernels do not take
  const int col_tiles = 1 << (a.qx + 1 - 8);                      // 256 real columns per tile
  const int row_tiles = 1 << (a.qy - ((variant & 2) ? 6 : 7));    // 64 or 128 rows per tile
  const int ntiles = col_tiles * row_tiles;
  dim3 grid((unsigned)((grid_cap > 0 && grid_cap < ntiles) ? grid_cap : ntiles), a.batch);
  const uint64_t r_bstride = a.r_batch > 1 ? a.r_plane_stride : 0;
  ProfScope prof(PROF_MERGE_GEMM, s);
#define CCUT_GEMM(E, R)                                                                                         \
  hipLaunchKernelGGL((k_merge_gemm<MODE, E, R>), grid, dim3(256), 0, s, a.Lhi, a.Llo, a.Rhi, a.Rlo, a.l_plane_stride, \
                     r_bstride, a.out, a.out_bstride * 2, a.qx, a.qy, S, col_tiles, row_tiles)
  switch (variant & 3) {
    case 0: CCUT_GEMM(0, 2); break;
    case 1: CCUT_GEMM(1, 2); break;
    case 2: CCUT_GEMM(0, 1); break;
    default: CCUT_GEMM(1, 1); break;
  }
#undef CCUT_GEMM
  CCUT_HIP(hipGetLastError());
  return 0;
}

}  // namespace

bool merge_mfma_supported(int qx, int qy) { return qx >= 7 && qy >= 7 && qx + 1 - 8 + qy - 7 <= 31; }

int launch_merge_mfma(const MergeMfmaArgs& a, int mode, int variant, int grid_cap, hipStream_t s) {
  if (!merge_mfma_supported(a.qx, a.qy)) return fail(CCUT_EUNSUPPORTED, "MFMA merge needs qx, qy >= 7");
  if (a.batch > 65535 || a.r_batch > 65535) return fail(CCUT_EUNSUPPORTED, "merge batch too large");
  switch (mode) {
    case MERGE_BF16X3: return launch_mode<MERGE_BF16X3>(a, variant, grid_cap, s);
    case MERGE_FP16X3: return launch_mode<MERGE_FP16X3>(a, variant, grid_cap, s);
    case MERGE_BF16: return launch_mode<MERGE_BF16>(a, variant, grid_cap, s);
    case MERGE_FP16X2: return launch_mode<MERGE_FP16X2>(a, variant, grid_cap, s);
    default: return fail(CCUT_EINVAL, "bad MFMA merge mode %d", mode);
  }
}

}  // namespace ccut
