// State-vector simulation kernel for gfx950 (Algorithm 2 of the paper, and
// the uncut baseline T_orig of Sec. III.A).
//
// A workgroup owns a block of 2^b amplitudes of one state: the amplitudes whose
// register qubits outside the pass group are fixed to the bits of the block id.
// The block is loaded into LDS (or generated as |0...0> on the first pass) and
// written back once.  When a state has at most 2^14 amplitudes the whole state
// is one block, so a subcircuit variant is simulated start to finish on chip
// and its final state is the only HBM traffic.  The low register qubits always
// belong to the group, so global loads and stores run over contiguous ranges.
//
// Inside the block the ops run in register stages: each thread takes the 16
// amplitudes spanned by the stage's four register bits, applies every op of
// the stage in registers (dense 2x2 gates on register bits, grouped so that a
// run of them costs one table read; diagonal phases, CZ parities and CX
// controls on any bit through each amplitude's known local index) and puts
// them back; one barrier per stage.  Blocks smaller than 2^9
// run their ops one at a time.  LDS is padded by one slot per 16 amplitudes
// so that strided stage accesses spread over the banks.
//
// On the MFMA path (blocks of at least 2^10 amplitudes, so that every lane of
// a wavefront holds a thread slot) a group (one 2x2 gate per register qubit, a
// 16x16 complex Kronecker product) is applied to a wavefront's 64 x 16 amplitudes as a real
// 32x32 by 32x64 product: two v_mfma_f32_32x32x16_f16 column tiles, each the
// sum of hi.hi + hi.lo + lo.hi products of float16 halves (float32 accumulate).
// The amplitudes stay in the lane that owns them: one lane-half swap puts the
// B operand in MFMA order and one more brings each column's 32 results back to
// its lane.  The state is scaled by 2^14 while a pass runs so that the low
// halves of typical amplitudes stay normal float16 numbers.
//
// A pass may start from another state than the one it writes (prefix sharing:
// a variant's chunk applied to its parent's state).
//
// One launch covers a list of jobs (state, pass, variant); a grid-stride loop
// over the job list makes the launch persistent when the grid is smaller than
// the work.
#include "ccut_internal.h"

#include <algorithm>

namespace ccut {

namespace {

constexpr int TAB = 128;  // offset-table entries per half (local bits 0..6 / 7..13)
constexpr int IO_BATCH = 2;  // amplitudes per thread in flight when a block is loaded (4 costs occupancy)
constexpr int R = 1 << REG_BITS;

__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ float2 cmadd2(float2 m0, float2 x, float2 m1, float2 y) {
  return make_float2(m0.x * x.x - m0.y * x.y + m1.x * y.x - m1.y * y.y,
                     m0.x * x.y + m0.y * x.x + m1.x * y.y + m1.y * y.x);
}

typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

// Swaps lanes 32..63 of x with lanes 0..31 of y.
__device__ __forceinline__ void swap_halves(uint32_t& x, uint32_t& y) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
  x = r[0];
  y = r[1];
}
__device__ __forceinline__ void swap_halves(float& x, float& y) {
  uint32_t u = __float_as_uint(x), v = __float_as_uint(y);
  swap_halves(u, v);
  x = __uint_as_float(u);
  y = __uint_as_float(v);
}

typedef __attribute__((ext_vector_type(2))) _Float16 f16x2;

// x - f32(half h) as one mixed-precision fma (h the low or high float16 of hp); exact,
// since x - round16(x) is representable in float32.  The compiler does not form
// v_fma_mix itself while float32 denormals are kept, so it is written out here.
__device__ __forceinline__ float sub_half_lo(uint32_t hp, float x) {
  float r;
  asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(hp), "v"(-1.0f), "v"(x));
  return r;
}
__device__ __forceinline__ float sub_half_hi(uint32_t hp, float x) {
  float r;
  asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(hp), "v"(-1.0f), "v"(x));
  return r;
}

// hi = float16(x), lo = float16(x - hi) for a pair, both rounded to nearest
// (v_cvt_pk_f16_f32: unbiased, so rounding errors do not drift the norm).
__device__ __forceinline__ void split_pair(float x0, float x1, uint32_t& hi, uint32_t& lo) {
  const f16x2 h = {(_Float16)x0, (_Float16)x1};
  hi = __builtin_bit_cast(uint32_t, h);
  const f16x2 l = {(_Float16)sub_half_lo(hi, x0), (_Float16)sub_half_hi(hi, x1)};
  lo = __builtin_bit_cast(uint32_t, l);
}

__device__ __forceinline__ f32x16 mfma16(const uint4& a, uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3,
                                         f32x16 c) {
  const uint4 b = make_uint4(b0, b1, b2, b3);
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                               0, 0);
}

// y = G x for every lane's 16 amplitudes (gt: this lane's four uint4 of the
// operand table, hi/lo for k-steps 0 (real parts) and 1 (imaginary parts)).
__device__ __forceinline__ void group_mfma(float2 (&a)[R], const uint4* __restrict__ gt) {
  const uint4 ghi0 = gt[0], ghi1 = gt[1], glo0 = gt[2], glo1 = gt[3];
  // B operand planes: element e of re / im, float16 hi and lo, two per dword
  uint32_t rh[8], rl[8], ih[8], il[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    split_pair(a[2 * j].x, a[2 * j + 1].x, rh[j], rl[j]);
    split_pair(a[2 * j].y, a[2 * j + 1].y, ih[j], il[j]);
  }
  // dwords 0..3 (elements 0..7) become the operand of column tile 0 (lanes 0..31),
  // dwords 4..7 (elements 8..15) that of tile 1 (lanes 32..63)
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    swap_halves(rh[j], rh[4 + j]);
    swap_halves(rl[j], rl[4 + j]);
    swap_halves(ih[j], ih[4 + j]);
    swap_halves(il[j], il[4 + j]);
  }
  f32x16 c0, c1;
#pragma unroll
  for (int v = 0; v < 16; ++v) c0[v] = c1[v] = 0.f;
  c0 = mfma16(glo0, rh[0], rh[1], rh[2], rh[3], c0);
  c0 = mfma16(ghi0, rl[0], rl[1], rl[2], rl[3], c0);
  c0 = mfma16(glo1, ih[0], ih[1], ih[2], ih[3], c0);
  c0 = mfma16(ghi1, il[0], il[1], il[2], il[3], c0);
  c0 = mfma16(ghi0, rh[0], rh[1], rh[2], rh[3], c0);
  c0 = mfma16(ghi1, ih[0], ih[1], ih[2], ih[3], c0);
  c1 = mfma16(glo0, rh[4], rh[5], rh[6], rh[7], c1);
  c1 = mfma16(ghi0, rl[4], rl[5], rl[6], rl[7], c1);
  c1 = mfma16(glo1, ih[4], ih[5], ih[6], ih[7], c1);
  c1 = mfma16(ghi1, il[4], il[5], il[6], il[7], c1);
  c1 = mfma16(ghi0, rh[4], rh[5], rh[6], rh[7], c1);
  c1 = mfma16(ghi1, ih[4], ih[5], ih[6], ih[7], c1);
  // accumulator v of a lane holds row (v & 3) + 4 (lane / 32) + 8 (v / 4) of its
  // tile's column lane % 32; after the swap c0[v] / c1[v] hold rows
  // (v & 3) + 8 (v / 4) and that + 4 of the lane's own column
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    float x = c0[v], y = c1[v];
    swap_halves(x, y);
    c0[v] = x;
    c1[v] = y;
  }
#pragma unroll
  for (int e = 0; e < R; ++e) {
    // rows 2 e (real part) and 2 e + 1 (imaginary part): registers v, v + 1 of c0 or c1
    const int v = 2 * (e & 1) + 4 * (e >> 2);
    a[e].x = ((e >> 1) & 1) ? c1[v] : c0[v];
    a[e].y = ((e >> 1) & 1) ? c1[v + 1] : c0[v + 1];
  }
}

template <int K>
__device__ __forceinline__ void dense_reg(float2 (&a)[R], const float* m) {
  const float2 m00 = make_float2(m[0], m[1]), m01 = make_float2(m[2], m[3]);
  const float2 m10 = make_float2(m[4], m[5]), m11 = make_float2(m[6], m[7]);
#pragma unroll
  for (int e = 0; e < R; ++e) {
    if (e & (1 << K)) continue;
    const float2 x = a[e], y = a[e | (1 << K)];
    a[e] = cmadd2(m00, x, m01, y);
    a[e | (1 << K)] = cmadd2(m10, x, m11, y);
  }
}

template <int K>
__device__ __forceinline__ void cx_reg(float2 (&a)[R], const int (&idx)[R], int c) {
#pragma unroll
  for (int e = 0; e < R; ++e) {
    if (e & (1 << K)) continue;
    if ((idx[e] >> c) & 1) {
      const float2 x = a[e];
      a[e] = a[e | (1 << K)];
      a[e | (1 << K)] = x;
    }
  }
}

// Matrix of a 2x2 record for this variant (slot alternative when the record has one).
__device__ __forceinline__ const float* kop_matrix(const KOp* k, int slot, int variant) {
  return k->m + ((slot >= 0) ? 8 * ((variant >> slot) & 1) : 0);
}

// First 32 bytes of a KOp (type, a, b, slot, cond, nterms, pad[0..1]): for a group
// they hold every member slot and the operand table index.
struct OpHead {
  int32_t type, a, b, slot, cond, nterms, pad0, pad1;
};

__device__ __forceinline__ OpHead load_head(const KOp* k) {
  const int4* p = reinterpret_cast<const int4*>(k);
  const int4 x = p[0], y = p[1];
  return OpHead{x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w};
}

// A header from the LDS copy: the same for every lane, so each field is moved to
// a scalar register (the interpreter branches on them).
__device__ __forceinline__ OpHead lds_head(const OpHead* p) {
  const int4* q = reinterpret_cast<const int4*>(p);
  const int4 x = q[0], y = q[1];
  return OpHead{__builtin_amdgcn_readfirstlane(x.x), __builtin_amdgcn_readfirstlane(x.y),
                __builtin_amdgcn_readfirstlane(x.z), __builtin_amdgcn_readfirstlane(x.w),
                __builtin_amdgcn_readfirstlane(y.x), __builtin_amdgcn_readfirstlane(y.y),
                __builtin_amdgcn_readfirstlane(y.z), __builtin_amdgcn_readfirstlane(y.w)};
}

// Operand table of a group or fused run for this variant: bit j of the choice is
// the variant bit of the j-th slot named in the header.
__device__ __forceinline__ int table_index(const OpHead& h, int variant) {
  const int slots[4] = {h.b, h.slot, h.cond, h.nterms};
  int sel = 0, j = 0;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    if (slots[p] >= 0) {
      sel |= ((variant >> slots[p]) & 1) << j;
      ++j;
    }
  }
  return h.pad0 + sel;
}

// Applies the ops [o0, o1) of a register stage to one thread's amplitudes.  The
// op headers come from the pass's copy in LDS (hdr[i] is op pass_op + i).
// full_waves: every lane of the wavefront holds a thread slot (the MFMA path
// exchanges data between lane halves, which needs both halves active).
template <bool MFMA>
__device__ __forceinline__ void run_stage_ops(float2 (&a)[R], const int (&idx)[R], const KOp* __restrict__ ops,
                                              const OpHead* hdr, int pass_op, int o0, int o1, uint64_t blockbase,
                                              int variant, const uint4* __restrict__ gtab, bool full_waves) {
  if (o0 >= o1) return;
  OpHead h = lds_head(hdr + (o0 - pass_op));
  for (int o = o0; o < o1;) {
    const KOp* k = ops + o;
    const int type = h.type;
    // operand-table path: a group, or a fused run (whose records are then skipped)
    const bool table = MFMA && full_waves && (type == KOP_GROUP || type == KOP_FUSED);
    const int next = o + (type == KOP_GROUP ? 1 + REG_BITS : (type == KOP_FUSED && table) ? 1 + h.a : 1);
    OpHead hn = h;
    if (next < o1) hn = lds_head(hdr + (next - pass_op));
    if (table) {
      const uint4* gt = gtab + (uint64_t)table_index(h, variant) * GROUP_TABLE_UINT4 + (threadIdx.x & 63) * 4;
      group_mfma(a, gt);
    } else if (type == KOP_FUSED) {
      // float32 path: the run's records follow and run one by one
    } else if (type == KOP_GROUP) {
      // one 2x2 gate per register position: every matrix address comes from the
      // header, the four matrices are fetched together, then straight-line arithmetic
      const float* m0 = kop_matrix(k + 1, h.b, variant);
      const float* m1 = kop_matrix(k + 2, h.slot, variant);
      const float* m2 = kop_matrix(k + 3, h.cond, variant);
      const float* m3 = kop_matrix(k + 4, h.nterms, variant);
      dense_reg<0>(a, m0);
      dense_reg<1>(a, m1);
      dense_reg<2>(a, m2);
      dense_reg<3>(a, m3);
    } else if (!(h.cond >= 0 && !((blockbase >> h.cond) & 1))) {
      const float* m = kop_matrix(k, h.slot, variant);
      if (type == KOP_DENSE) {
        switch (h.a) {
          case 0: dense_reg<0>(a, m); break;
          case 1: dense_reg<1>(a, m); break;
          case 2: dense_reg<2>(a, m); break;
          default: dense_reg<3>(a, m); break;
        }
      } else if (type == KOP_DIAG) {
        const int jb = h.a;
        const float2 d0 = make_float2(m[0], m[1]), d1 = make_float2(m[6], m[7]);
#pragma unroll
        for (int e = 0; e < R; ++e) a[e] = cmul(((idx[e] >> jb) & 1) ? d1 : d0, a[e]);
      } else if (type == KOP_CZL) {
        // terms outside, amplitudes inside: each (shift, mask) pair is read once, not
        // once per amplitude (a scalar load and its wait each time); popcounts are
        // summed (only the parity is used), which folds into the count instruction
        const uint32_t* t = reinterpret_cast<const uint32_t*>(k->m);
        uint32_t par[R];
#pragma unroll
        for (int e = 0; e < R; ++e) par[e] = 0;
        for (int q = 0; q < h.nterms; ++q) {
          // terms 0 and 1 come with the header
          const uint32_t sh = q == 0 ? (uint32_t)h.a : q == 1 ? (uint32_t)h.pad0 : t[2 * q];
          const uint32_t mk = q == 0 ? (uint32_t)h.b : q == 1 ? (uint32_t)h.pad1 : t[2 * q + 1];
#pragma unroll
          for (int e = 0; e < R; ++e) {
            const uint32_t i = (uint32_t)idx[e];
            par[e] += __popc(i & (i >> sh) & mk);
          }
        }
        // negate on odd parity: bit 0 of the count shifted into both sign bits
#pragma unroll
        for (int e = 0; e < R; ++e) {
          const uint32_t sgn = par[e] << 31;
          a[e].x = __uint_as_float(__float_as_uint(a[e].x) ^ sgn);
          a[e].y = __uint_as_float(__float_as_uint(a[e].y) ^ sgn);
        }
      } else if (type == KOP_SCALAR) {
        const bool bit = (blockbase >> h.a) & 1;
        const float2 ph = bit ? make_float2(m[6], m[7]) : make_float2(m[0], m[1]);
#pragma unroll
        for (int e = 0; e < R; ++e) a[e] = cmul(ph, a[e]);
      } else {  // KOP_CXL: control local bit a, target register position b
        switch (h.b) {
          case 0: cx_reg<0>(a, idx, h.a); break;
          case 1: cx_reg<1>(a, idx, h.a); break;
          case 2: cx_reg<2>(a, idx, h.a); break;
          default: cx_reg<3>(a, idx, h.a); break;
        }
      }
    }
    h = hn;
    o = next;
  }
}

template <int NT>
__device__ __forceinline__ void run_ops_direct(float2* sh, int nb, const KOp* __restrict__ ops, int o0, int o1,
                                               uint64_t blockbase, int variant) {
  const int tid = threadIdx.x;
  for (int o = o0; o < o1; ++o) {
    const KOp* k = ops + o;
    const int cond = k->cond;
    if (cond >= 0 && !((blockbase >> cond) & 1)) continue;
    const int slot = k->slot;
    const float* m = k->m + ((slot >= 0) ? 8 * ((variant >> slot) & 1) : 0);
    const int type = k->type;
    if (type == KOP_DENSE || type == KOP_DIAG || type == KOP_CXL) {
      const int j = type == KOP_CXL ? k->b : k->a;
      const int low = (1 << j) - 1;
      const float2 m00 = make_float2(m[0], m[1]), m01 = make_float2(m[2], m[3]);
      const float2 m10 = make_float2(m[4], m[5]), m11 = make_float2(m[6], m[7]);
      for (int p = tid; p < (nb >> 1); p += NT) {
        const int i0 = ((p & ~low) << 1) | (p & low);
        const int i1 = i0 | (1 << j);
        const float2 x = sh[pad(i0)], y = sh[pad(i1)];
        if (type == KOP_DENSE) {
          sh[pad(i0)] = cmadd2(m00, x, m01, y);
          sh[pad(i1)] = cmadd2(m10, x, m11, y);
        } else if (type == KOP_DIAG) {
          sh[pad(i0)] = cmul(m00, x);
          sh[pad(i1)] = cmul(m11, y);
        } else if ((i0 >> k->a) & 1) {
          sh[pad(i0)] = y;
          sh[pad(i1)] = x;
        }
      }
    } else if (type == KOP_CZL) {
      const uint32_t* t = reinterpret_cast<const uint32_t*>(k->m);
      const int nt = k->nterms;
      for (int i = tid; i < nb; i += NT) {
        uint32_t par = 0;
        for (int q = 0; q < nt; ++q) par ^= __popc((uint32_t)i & ((uint32_t)i >> t[2 * q]) & t[2 * q + 1]);
        if (par & 1) {
          const float2 v = sh[pad(i)];
          sh[pad(i)] = make_float2(-v.x, -v.y);
        }
      }
    } else {  // KOP_SCALAR
      const bool bit = (blockbase >> k->a) & 1;
      const float2 ph = bit ? make_float2(m[6], m[7]) : make_float2(m[0], m[1]);
      for (int i = tid; i < nb; i += NT) sh[pad(i)] = cmul(ph, sh[pad(i)]);
    }
    __syncthreads();
  }
}

// Index of the last job whose first workgroup is <= wg (jobs sorted by wg_begin):
// a 64-ary search, one round of vector loads per level instead of a chain of
// dependent scalar loads.  Every wavefront of the workgroup runs it.
__device__ __forceinline__ int find_job(const SimJob* __restrict__ jobs, int n_jobs, int wg) {
  const int lane = threadIdx.x & 63;
  int lo = 0, n = n_jobs;  // the job lies in [lo, lo + n)
  while (n > 1) {
    const int step = (n + 63) >> 6;
    const bool ok = lane * step < n && jobs[lo + lane * step].wg_begin <= wg;
    const uint64_t m = __ballot(ok);  // lanes 0..i: wg_begin is non-decreasing
    const int i = 63 - __builtin_clzll(m);
    lo += i * step;
    n = min(step, n - i * step);
  }
  return lo;
}

// First 32 bytes of a StageDesc: op range and register bits.
struct StageHead {
  int32_t op_begin, op_count, reg[REG_BITS], pad[2];
};

// rec_cap: LDS room (32-byte records) for the op headers and stage heads of the
// largest pass of the launch; a pass's stage heads follow its own op headers.
// At most 128 VGPRs (four wavefronts per SIMD): two 512-thread workgroups share a
// compute unit where their LDS allows it, one computing while the other waits.
template <int NT, bool MFMA>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_sim(const SimJob* __restrict__ jobs, int n_jobs, int total_wg,
                                            int wg_offset, const PassDesc* __restrict__ passes,
                                            const StageDesc* __restrict__ stages, const KOp* __restrict__ ops,
                                            const uint4* __restrict__ gtab, float2* __restrict__ base,
                                            int rec_cap) {
  const float scale_in = MFMA ? SIM_MFMA_SCALE : 1.0f, scale_out = MFMA ? 1.0f / SIM_MFMA_SCALE : 1.0f;
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* lo_tab = reinterpret_cast<uint64_t*>(smem);
  uint64_t* hi_tab = lo_tab + TAB;
  OpHead* hdr = reinterpret_cast<OpHead*>(hi_tab + TAB);
  float2* sh = reinterpret_cast<float2*>(hdr + rec_cap);
  const int tid = threadIdx.x;

  for (int w = blockIdx.x; w < total_wg; w += gridDim.x) {
    const int wg = w + wg_offset;
    // the same index in every lane: readfirstlane lets the compiler keep the job in scalar registers
    const SimJob job = jobs[n_jobs > 1 ? __builtin_amdgcn_readfirstlane(find_job(jobs, n_jobs, wg)) : 0];
    const PassDesc* P = passes + job.pass_id;
    StageHead* stg = reinterpret_cast<StageHead*>(hdr + P->op_count);  // after the pass's op headers
    const int b = P->b;
    const int nb = 1 << b;
    const int nfix = P->nq - b;
    const uint32_t blk = (uint32_t)(wg - job.wg_begin);
    uint64_t blockbase = 0;
    for (int j = 0; j < nfix; ++j) blockbase |= (uint64_t)((blk >> j) & 1u) << P->fixed[j];
    float2* st = base + job.state_off;
    const float2* src = P->from_src ? base + job.src_off : st;  // prefix sharing: the parent state

    // offset tables: scatter of local bits 0..6 and 7..b-1 into register positions
    const int blo = b < 7 ? b : 7;
    for (int t = tid; t < 2 * TAB; t += NT) {
      uint64_t off = 0;
      if (t < TAB) {
        for (int j = 0; j < blo; ++j) off |= (uint64_t)((t >> j) & 1) << P->group[j];
        lo_tab[t] = off;
      } else {
        int u = t - TAB;
        for (int j = 0; j < b - 7; ++j) off |= (uint64_t)((u >> j) & 1) << P->group[7 + j];
        hi_tab[u] = off;
      }
    }
    // the pass's op headers and stage heads, copied to LDS in one burst: the stages
    // then read them without a scalar-cache miss each (one workgroup per compute
    // unit finds nothing of them cached)
    if (P->stage_count > 0) {
      for (int t = tid; t < P->op_count; t += NT) hdr[t] = load_head(ops + P->op_begin + t);
      for (int t = tid; t < P->stage_count; t += NT) {
        const int4* q = reinterpret_cast<const int4*>(stages + P->stage_begin + t);
        int4* d = reinterpret_cast<int4*>(stg + t);
        d[0] = q[0];
        d[1] = q[1];
      }
    }
    __syncthreads();

    if (P->init) {
      for (int i = tid; i < nb; i += NT) sh[pad(i)] = make_float2(0.f, 0.f);
      __syncthreads();
      if (tid == 0 && blockbase == 0) sh[0] = make_float2(scale_in, 0.f);
    } else {
      // IO_BATCH amplitudes per thread at a time: their offsets are read from the
      // tables first, then all their loads are issued, then they are written to LDS
      // (one at a time, every table read waits behind the previous LDS write and every
      // load for its table reads: one L2 or HBM latency per amplitude)
      for (int i0 = tid; i0 < nb; i0 += IO_BATCH * NT) {
        uint64_t off[IO_BATCH];
        float2 v[IO_BATCH];
#pragma unroll
        for (int u = 0; u < IO_BATCH; ++u) {
          const int i = i0 + u * NT;
          off[u] = i < nb ? lo_tab[i & (TAB - 1)] + hi_tab[i >> 7] : 0;
        }
#pragma unroll
        for (int u = 0; u < IO_BATCH; ++u)
          if (i0 + u * NT < nb) v[u] = src[blockbase + off[u]];
#pragma unroll
        for (int u = 0; u < IO_BATCH; ++u) {
          const int i = i0 + u * NT;
          if (i < nb) sh[pad(i)] = make_float2(v[u].x * scale_in, v[u].y * scale_in);
        }
      }
    }
    __syncthreads();

    if (P->stage_count == 0) {
      run_ops_direct<NT>(sh, nb, ops, P->op_begin, P->op_begin + P->op_count, blockbase, job.variant);
    } else {
      const int active = nb >> REG_BITS;  // thread slots per stage
      for (int si = 0; si < P->stage_count; ++si) {
        const StageDesc* S = stages + P->stage_begin + si;
        const int4* sq = reinterpret_cast<const int4*>(stg + si);
        const int4 s0 = sq[0], s1 = sq[1];
        const int op_begin = __builtin_amdgcn_readfirstlane(s0.x), op_count = __builtin_amdgcn_readfirstlane(s0.y);
        const int reg[REG_BITS] = {__builtin_amdgcn_readfirstlane(s0.z), __builtin_amdgcn_readfirstlane(s0.w),
                                   __builtin_amdgcn_readfirstlane(s1.x), __builtin_amdgcn_readfirstlane(s1.y)};
        for (int tt = tid; tt < active; tt += NT) {
          // insert a zero at each register bit (ascending) to get the thread's base index
          int tb = tt;
#pragma unroll
          for (int k = 0; k < REG_BITS; ++k) {
            const int r = reg[k];
            tb = ((tb >> r) << (r + 1)) | (tb & ((1 << r) - 1));
          }
          const int pb = pad(tb);
          int idx[R];
          float2 a[R];
#pragma unroll
          for (int e = 0; e < R; ++e) {
            idx[e] = tb | S->roff[e];
            a[e] = sh[pb + S->proff[e]];
          }
          run_stage_ops<MFMA>(a, idx, ops, hdr, P->op_begin, op_begin, op_begin + op_count, blockbase, job.variant,
                              gtab, (active & 63) == 0);
#pragma unroll
          for (int e = 0; e < R; ++e) sh[pb + S->proff[e]] = a[e];
        }
        __syncthreads();
      }
    }

    for (int i = tid; i < nb; i += NT) {
      const float2 v = sh[pad(i)];
      st[blockbase + lo_tab[i & (TAB - 1)] + hi_tab[i >> 7]] = make_float2(v.x * scale_out, v.y * scale_out);
    }
    __syncthreads();
  }
}

// Copies a table image from pinned host memory (the staging ring) into the arena.
// A kernel reading host memory over the bus starts sooner than a copy-engine
// transfer, and the images are small (tens to hundreds of KiB).
__global__ __launch_bounds__(256) void k_table_copy(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                    uint64_t n16) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (uint64_t)gridDim.x * 256)
    dst[i] = src[i];
}

static_assert(sizeof(OpHead) == sizeof(StageHead), "one LDS record size");
constexpr size_t shmem_bytes(int bmax, int rec_cap) {
  return 2 * TAB * sizeof(uint64_t) + (size_t)rec_cap * sizeof(OpHead) +
         sizeof(float2) * (((size_t)1 << bmax) + ((size_t)1 << bmax) / 16);
}

// ---- operand tables: the 16x16 matrix of a group or fused run

__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Applies one record of a fused run to the matrix G[row][col] held in LDS (float64),
// every lane taking its share of the rows and columns.  Amplitude index e has bit p
// of e at register position p (local bit lb[p]).  hdr: the slot fields of the run's
// header (bit j of the table choice sel is the j-th non-negative one).  The caller
// orders consecutive records with a barrier.
__device__ __forceinline__ void fused_apply(const KOp* __restrict__ k, double2 (*G)[R + 1], const int (&hdr)[REG_BITS], int sel,
                            const int (&lb)[REG_BITS], int lane) {
  int bit = 0;
  if (k->slot >= 0) {
    int j = 0;
#pragma unroll
    for (int p = 0; p < REG_BITS; ++p) {
      if (hdr[p] >= 0) {
        if (hdr[p] == k->slot) bit = (sel >> j) & 1;
        ++j;
      }
    }
  }
  const float* m = k->m + 8 * bit;
  auto pos = [&](int local) {
    int p = 0;
#pragma unroll
    for (int q = 0; q < REG_BITS; ++q)
      if (lb[q] == local) p = q;
    return p;
  };
  const int type = k->type;
  if (type == KOP_DENSE || type == KOP_CXL) {
    // 8 row pairs x 16 columns: two (pair, column) units per lane
    const int p = type == KOP_DENSE ? k->a : k->b;
    const int pc = type == KOP_CXL ? pos(k->a) : 0;
    const double2 m00 = make_double2(m[0], m[1]), m01 = make_double2(m[2], m[3]);
    const double2 m10 = make_double2(m[4], m[5]), m11 = make_double2(m[6], m[7]);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int u = lane + 64 * i, col = u & 15, t = u >> 4;
      const int e0 = ((t >> p) << (p + 1)) | (t & ((1 << p) - 1)), e1 = e0 | (1 << p);
      const double2 x = G[e0][col], y = G[e1][col];
      if (type == KOP_DENSE) {
        G[e0][col] = dadd(dmul(m00, x), dmul(m01, y));
        G[e1][col] = dadd(dmul(m10, x), dmul(m11, y));
      } else if ((e0 >> pc) & 1) {
        G[e0][col] = y;
        G[e1][col] = x;
      }
    }
  } else if (type == KOP_DIAG || type == KOP_CZL) {
    // 256 entries: four per lane
    const int pd = type == KOP_DIAG ? pos(k->a) : 0;
    const double2 d0 = make_double2(m[0], m[1]), d1 = make_double2(m[6], m[7]);
    const uint32_t* t = reinterpret_cast<const uint32_t*>(k->m);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int u = lane + 64 * i, row = u >> 4, col = u & 15;
      if (type == KOP_DIAG) {
        G[row][col] = dmul(((row >> pd) & 1) ? d1 : d0, G[row][col]);
      } else {
        uint32_t li = 0;
#pragma unroll
        for (int q = 0; q < REG_BITS; ++q) li |= (uint32_t)((row >> q) & 1) << lb[q];
        uint32_t par = 0;
        for (int q = 0; q < k->nterms; ++q) par += __popc(li & (li >> t[2 * q]) & t[2 * q + 1]);
        if (par & 1) G[row][col] = make_double2(-G[row][col].x, -G[row][col].y);
      }
    }
  }
  // a group header inside the run: its member records follow
}

// One wavefront per (group or fused run, slot choice); lane l writes its four
// uint4 of the real 32x32 A operand (row m = l % 32, columns 16 s + 8 (l / 32) + e):
// hi and lo float16 parts, rounded to nearest.  A group's entries are products of
// its four 2x2 matrices (float32, each lane its own); a fused run's matrix is
// composed in LDS (float64), its records staged in LDS and applied in order to
// the identity.
__global__ __launch_bounds__(64) void k_group_tables(const KOp* __restrict__ ops, const GroupRef* __restrict__ refs,
                                                     uint4* __restrict__ gtab) {
  __shared__ double2 G[R][R + 1];  // G[row][col]
  __shared__ __align__(16) KOp recs[FUSED_MAX_RECORDS];
  const GroupRef ref = refs[blockIdx.x];
  const KOp* g = ops + ref.op;
  const int lane = threadIdx.x;
  const int m = lane & 31, h = lane >> 5;
  // output rows interleaved: row 2 e = Re y_e, row 2 e + 1 = Im y_e, so that each
  // amplitude's two parts land in adjacent accumulator registers
  const int row = m >> 1;
  const bool imag_row = m & 1;
  uint32_t hi[2][4], lo[2][4];
  // entries (A[m][16 st + 8 h + c], c and c + 1) to float16 hi / lo pairs
  auto pack = [&](int st, int c, double v0, double v1) {
    const _Float16 h0 = (_Float16)(float)v0, h1 = (_Float16)(float)v1;
    const _Float16 l0 = (_Float16)(float)(v0 - (double)h0), l1 = (_Float16)(float)(v1 - (double)h1);
    hi[st][c / 2] = (uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
    lo[st][c / 2] = (uint32_t)__builtin_bit_cast(uint16_t, l0) | ((uint32_t)__builtin_bit_cast(uint16_t, l1) << 16);
  };
  // row 2 e: Re y = Re G Re x - Im G Im x;  row 2 e + 1: Im y = Im G Re x + Re G Im x
  if (g->type == KOP_FUSED) {
    const int hdr[REG_BITS] = {g->b, g->slot, g->cond, g->nterms};
    const int32_t* bits = reinterpret_cast<const int32_t*>(g->m);
    int lb[REG_BITS];
#pragma unroll
    for (int p = 0; p < REG_BITS; ++p) lb[p] = bits[p];
    const int n = g->a;
    constexpr int U4 = (int)(sizeof(KOp) / 16);
    for (int i = lane; i < n * U4; i += 64)
      reinterpret_cast<uint4*>(recs)[i] = reinterpret_cast<const uint4*>(g + 1)[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int u = lane + 64 * i;
      G[u >> 4][u & 15] = make_double2((u >> 4) == (u & 15) ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    for (int r = 0; r < n; ++r) {
      fused_apply(recs + r, G, hdr, ref.sel, lb, lane);
      __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < 8; c += 2) {
      const double2 g0 = G[row][8 * h + c], g1 = G[row][8 * h + c + 1];
      pack(0, c, imag_row ? g0.y : g0.x, imag_row ? g1.y : g1.x);
      pack(1, c, imag_row ? g0.x : -g0.y, imag_row ? g1.x : -g1.y);
    }
  } else {
    // 2x2 matrix of position p for this slot choice, in LDS: u[p][2 * row + col]
    // (read below at lane-dependent indices)
    __shared__ float2 u[REG_BITS][4];
    if (lane < 16) {
      const int p = lane >> 2, t = lane & 3;
      int j = 0;
#pragma unroll
      for (int q = 0; q < REG_BITS; ++q) j += q < p && g[1 + q].slot >= 0;
      const KOp* k = g + 1 + p;
      const int bit = k->slot >= 0 ? (ref.sel >> j) & 1 : 0;
      u[p][t] = make_float2(k->m[8 * bit + 2 * t], k->m[8 * bit + 2 * t + 1]);
    }
    __syncthreads();
    auto entry = [&](int col) {
      float2 gv = make_float2(1.f, 0.f);
#pragma unroll
      for (int p = 0; p < 4; ++p) gv = cmul(gv, u[p][2 * ((row >> p) & 1) + ((col >> p) & 1)]);
      return gv;
    };
#pragma unroll
    for (int c = 0; c < 8; c += 2) {
      const float2 g0 = entry(8 * h + c), g1 = entry(8 * h + c + 1);
      pack(0, c, imag_row ? g0.y : g0.x, imag_row ? g1.y : g1.x);
      pack(1, c, imag_row ? g0.x : -g0.y, imag_row ? g1.x : -g1.y);
    }
  }
  uint4* out = gtab + (uint64_t)blockIdx.x * GROUP_TABLE_UINT4 + lane * 4;
  out[0] = make_uint4(hi[0][0], hi[0][1], hi[0][2], hi[0][3]);
  out[1] = make_uint4(hi[1][0], hi[1][1], hi[1][2], hi[1][3]);
  out[2] = make_uint4(lo[0][0], lo[0][1], lo[0][2], lo[0][3]);
  out[3] = make_uint4(lo[1][0], lo[1][1], lo[1][2], lo[1][3]);
}

template <int NT, bool MFMA>
int launch_sim_t(const SimJob* d_jobs, int n_jobs, int total_wg, int wg_offset, const PassDesc* d_passes,
                 const StageDesc* d_stages, const KOp* d_ops, const uint4* gtab, float* base, int bmax, int rec_cap,
                 int grid, hipStream_t s) {
  const size_t shmem = shmem_bytes(bmax, rec_cap);
  static bool attr_set = false;
  if (!attr_set) {
    CCUT_HIP(hipFuncSetAttribute((const void*)k_sim<NT, MFMA>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)SIM_LDS_MAX));
    attr_set = true;
  }
  ProfScope prof(PROF_SIM, s);
  hipLaunchKernelGGL((k_sim<NT, MFMA>), dim3(grid), dim3(NT), shmem, s, d_jobs, n_jobs, total_wg, wg_offset,
                     d_passes, d_stages, d_ops, gtab, reinterpret_cast<float2*>(base), rec_cap);
  CCUT_HIP(hipGetLastError());
  return 0;
}

template <bool MFMA>
int launch_sim_m(const SimJob* d_jobs, int n_jobs, int total_wg, int wg_offset, const PassDesc* d_passes,
                 const StageDesc* d_stages, const KOp* d_ops, const uint4* gtab, float* base, int bmax, int rec_cap,
                 int threads, int grid, hipStream_t s) {
  switch (threads) {
    case 256:
      return launch_sim_t<256, MFMA>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_stages, d_ops, gtab, base,
                                     bmax, rec_cap, grid, s);
    case 512:
      return launch_sim_t<512, MFMA>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_stages, d_ops, gtab, base,
                                     bmax, rec_cap, grid, s);
    case 1024:
      return launch_sim_t<1024, MFMA>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_stages, d_ops, gtab, base,
                                      bmax, rec_cap, grid, s);
    default:
      return fail(CCUT_EINVAL, "unsupported workgroup size %d", threads);
  }
}

}  // namespace

size_t sim_shmem_bytes(int bmax, int rec_cap) { return shmem_bytes(bmax, rec_cap); }

int launch_sim(const SimJob* d_jobs, int n_jobs, int total_wg, int wg_offset, const PassDesc* d_passes,
               const StageDesc* d_stages, const KOp* d_ops, const uint4* gtab, float* base, int bmax, int rec_cap,
               int threads, int grid_cap, hipStream_t s) {
  if (total_wg <= 0 || n_jobs <= 0) return 0;
  if (bmax < 1 || bmax > PASS_MAX_B) return fail(CCUT_EINVAL, "bad block bits %d", bmax);
  if (rec_cap < 0 || shmem_bytes(bmax, rec_cap) > SIM_LDS_MAX)
    return fail(CCUT_EUNSUPPORTED, "simulation pass needs %zu bytes of LDS (at most %zu)",
                shmem_bytes(bmax, rec_cap), (size_t)SIM_LDS_MAX);
  const int grid = (grid_cap > 0 && grid_cap < total_wg) ? grid_cap : total_wg;
  if (gtab)
    return launch_sim_m<true>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_stages, d_ops, gtab, base, bmax,
                              rec_cap, threads, grid, s);
  return launch_sim_m<false>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_stages, d_ops, nullptr, base, bmax,
                             rec_cap, threads, grid, s);
}

int launch_table_copy(void* dst, const void* host_src, uint64_t bytes, hipStream_t s) {
  if ((bytes & 15) || ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(host_src)) & 15))
    return fail(CCUT_EINVAL, "table copy needs 16-byte alignment");
  const uint64_t n16 = bytes / 16;
  const uint64_t blocks = std::min<uint64_t>((n16 + 255) / 256, 1024);
  if (blocks == 0) return 0;
  ProfScope prof(PROF_TABLES, s);
  hipLaunchKernelGGL(k_table_copy, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint4*>(dst),
                     static_cast<const uint4*>(host_src), n16);
  CCUT_HIP(hipGetLastError());
  return 0;
}

int launch_group_tables(const KOp* d_ops, const GroupRef* d_refs, int n, uint4* gtab, hipStream_t s) {
  if (n <= 0) return 0;
  ProfScope prof(PROF_TABLES, s);
  hipLaunchKernelGGL(k_group_tables, dim3(n), dim3(64), 0, s, d_ops, d_refs, gtab);
  CCUT_HIP(hipGetLastError());
  return 0;
}

}  // namespace ccut
