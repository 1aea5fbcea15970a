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

// y = G x for every lane's 16 amplitudes (the group's operand table gt: this
// lane's four uint4, hi/lo for k-steps 0 (real parts) and 1 (imaginary parts)).
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

// Applies the ops [o0, o1) of a register stage to one thread's amplitudes.  The
// next op's header is loaded before the current op runs, so its load latency
// (op tables are read by every workgroup) hides behind the arithmetic.
// full_waves: every lane of the wavefront holds a thread slot (the MFMA path
// exchanges data between lane halves, which needs both halves active).
template <bool MFMA>
__device__ __forceinline__ void run_stage_ops(float2 (&a)[R], const int (&idx)[R], const KOp* __restrict__ ops,
                                              int o0, int o1, uint64_t blockbase, int variant,
                                              const uint4* __restrict__ gtab, bool full_waves) {
  if (o0 >= o1) return;
  OpHead h = load_head(ops + o0);
  for (int o = o0; o < o1;) {
    const KOp* k = ops + o;
    const int type = h.type;
    const int next = o + (type == KOP_GROUP ? 1 + REG_BITS : 1);
    OpHead hn = h;
    if (next < o1) hn = load_head(ops + next);
    if (MFMA && full_waves && type == KOP_GROUP) {
      // table of this choice of the members' slots: bit j = slot bit of the j-th slotted member
      const int slots[4] = {h.b, h.slot, h.cond, h.nterms};
      int sel = 0, j = 0;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        if (slots[p] >= 0) {
          sel |= ((variant >> slots[p]) & 1) << j;
          ++j;
        }
      }
      const uint4* gt = gtab + (uint64_t)(h.pad0 + sel) * GROUP_TABLE_UINT4 + (threadIdx.x & 63) * 4;
      group_mfma(a, gt);
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
          const uint32_t sh = t[2 * q], mk = t[2 * q + 1];
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

template <int NT, bool MFMA>
__global__ __launch_bounds__(NT) void k_sim(const SimJob* __restrict__ jobs, int n_jobs, int total_wg,
                                            int wg_offset, const PassDesc* __restrict__ passes,
                                            const StageDesc* __restrict__ stages, const KOp* __restrict__ ops,
                                            const uint4* __restrict__ gtab, float2* __restrict__ base) {
  const float scale_in = MFMA ? SIM_MFMA_SCALE : 1.0f, scale_out = MFMA ? 1.0f / SIM_MFMA_SCALE : 1.0f;
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* lo_tab = reinterpret_cast<uint64_t*>(smem);
  uint64_t* hi_tab = lo_tab + TAB;
  float2* sh = reinterpret_cast<float2*>(hi_tab + TAB);
  const int tid = threadIdx.x;

  for (int w = blockIdx.x; w < total_wg; w += gridDim.x) {
    const int wg = w + wg_offset;
    // job lookup: last job whose first workgroup is <= wg
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].wg_begin <= wg) lo = mid; else hi = mid - 1;
    }
    const SimJob job = jobs[lo];
    const PassDesc* P = passes + job.pass_id;
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
        for (int tt = tid; tt < active; tt += NT) {
          // insert a zero at each register bit (ascending) to get the thread's base index
          int tb = tt;
#pragma unroll
          for (int k = 0; k < REG_BITS; ++k) {
            const int r = S->reg[k];
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
          run_stage_ops<MFMA>(a, idx, ops, S->op_begin, S->op_begin + S->op_count, blockbase, job.variant, gtab,
                              (active & 63) == 0);
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

constexpr size_t shmem_bytes(int bmax) {
  return 2 * TAB * sizeof(uint64_t) + sizeof(float2) * (((size_t)1 << bmax) + ((size_t)1 << bmax) / 16);
}

// One wavefront per (group, slot choice): lane l writes its four uint4 of the
// real 32x32 A operand (row m = l % 32, columns 16 s + 8 (l / 32) + e).
__global__ __launch_bounds__(64) void k_group_tables(const KOp* __restrict__ ops, const GroupRef* __restrict__ refs,
                                                     uint4* __restrict__ gtab) {
  const GroupRef ref = refs[blockIdx.x];
  const KOp* g = ops + ref.op;
  const int lane = threadIdx.x;
  // 2x2 matrix of position p for this slot choice: u[p][2 * row + col]
  float2 u[4][4];
  int j = 0;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const KOp* k = g + 1 + p;
    int bit = 0;
    if (k->slot >= 0) {
      bit = (ref.sel >> j) & 1;
      ++j;
    }
    const float* m = k->m + 8 * bit;
#pragma unroll
    for (int t = 0; t < 4; ++t) u[p][t] = make_float2(m[2 * t], m[2 * t + 1]);
  }
  const int m = lane & 31, h = lane >> 5;
  // output rows interleaved: row 2 e = Re y_e, row 2 e + 1 = Im y_e, so that each
  // amplitude's two parts land in adjacent accumulator registers
  const int row = m >> 1;
  const bool imag_row = m & 1;
  uint32_t hi[2][4], lo[2][4];
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    float v0[2], v1[2];  // [k-step]
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int col = 8 * h + e + d;
      float2 gv = make_float2(1.f, 0.f);
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const bool rb = (row >> p) & 1, cb = (col >> p) & 1;  // selects, no indexed register array
        const float2 f = rb ? (cb ? u[p][3] : u[p][2]) : (cb ? u[p][1] : u[p][0]);
        gv = cmul(gv, f);
      }
      // row 2 e: Re y = Re G Re x - Im G Im x;  row 2 e + 1: Im y = Im G Re x + Re G Im x
      const float s0 = imag_row ? gv.y : gv.x;
      const float s1 = imag_row ? gv.x : -gv.y;
      if (d == 0) { v0[0] = s0; v0[1] = s1; } else { v1[0] = s0; v1[1] = s1; }
    }
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      // float16 hi / lo of the float32 products: round to nearest for the table
      const _Float16 h0 = (_Float16)v0[st], h1 = (_Float16)v1[st];
      const _Float16 l0 = (_Float16)(v0[st] - (float)h0), l1 = (_Float16)(v1[st] - (float)h1);
      hi[st][e / 2] = (uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
      lo[st][e / 2] = (uint32_t)__builtin_bit_cast(uint16_t, l0) | ((uint32_t)__builtin_bit_cast(uint16_t, l1) << 16);
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
                 const StageDesc* d_stages, const KOp* d_ops, const uint4* gtab, float* base, int bmax, int grid,
                 hipStream_t s) {
  const size_t shmem = shmem_bytes(bmax);
  static bool attr_set = false;
  if (!attr_set) {
    CCUT_HIP(hipFuncSetAttribute((const void*)k_sim<NT, MFMA>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)shmem_bytes(PASS_MAX_B)));
    attr_set = true;
  }
  ProfScope prof(PROF_SIM, s);
  hipLaunchKernelGGL((k_sim<NT, MFMA>), dim3(grid), dim3(NT), shmem, s, d_jobs, n_jobs, total_wg, wg_offset,
                     d_passes, d_stages, d_ops, gtab, reinterpret_cast<float2*>(base));
  CCUT_HIP(hipGetLastError());
  return 0;
}

template <bool MFMA>
int launch_sim_m(const SimJob* d_jobs, int n_jobs, int total_wg, int wg_offset, const PassDesc* d_passes,
                 const StageDesc* d_stages, const KOp* d_ops, const uint4* gtab, float* base, int bmax,
                 int threads, int grid, hipStream_t s) {
  switch (threads) {
    case 256:
      return launch_sim_t<256, MFMA>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_stages, d_ops, gtab, base,
                                     bmax, grid, s);
    case 512:
      return launch_sim_t<512, MFMA>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_stages, d_ops, gtab, base,
                                     bmax, grid, s);
    case 1024:
      return launch_sim_t<1024, MFMA>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_stages, d_ops, gtab, base,
                                      bmax, grid, s);
    default:
      return fail(CCUT_EINVAL, "unsupported workgroup size %d", threads);
  }
}

}  // namespace

int launch_sim(const SimJob* d_jobs, int n_jobs, int total_wg, int wg_offset, const PassDesc* d_passes,
               const StageDesc* d_stages, const KOp* d_ops, const uint4* gtab, float* base, int bmax, int threads,
               int grid_cap, hipStream_t s) {
  if (total_wg <= 0 || n_jobs <= 0) return 0;
  if (bmax < 1 || bmax > PASS_MAX_B) return fail(CCUT_EINVAL, "bad block bits %d", bmax);
  const int grid = (grid_cap > 0 && grid_cap < total_wg) ? grid_cap : total_wg;
  if (gtab)
    return launch_sim_m<true>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_stages, d_ops, gtab, base, bmax,
                              threads, grid, s);
  return launch_sim_m<false>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_stages, d_ops, nullptr, base, bmax,
                             threads, grid, s);
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
