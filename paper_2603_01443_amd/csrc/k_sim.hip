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
// One launch covers a list of jobs (state, pass, variant); a grid-stride loop
// over the job list makes the launch persistent when the grid is smaller than
// the work.
#include "ccut_internal.h"

namespace ccut {

namespace {

constexpr int TAB = 128;  // offset-table entries per half (local bits 0..6 / 7..13)
constexpr int R = 1 << REG_BITS;

__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ float2 cmadd2(float2 m0, float2 x, float2 m1, float2 y) {
  return make_float2(m0.x * x.x - m0.y * x.y + m1.x * y.x - m1.y * y.y,
                     m0.x * x.y + m0.y * x.x + m1.x * y.y + m1.y * y.x);
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

// Applies the ops [o0, o1) of a register stage to one thread's amplitudes.
__device__ __forceinline__ void run_stage_ops(float2 (&a)[R], const int (&idx)[R], const KOp* __restrict__ ops,
                                              int o0, int o1, uint64_t blockbase, int variant) {
  for (int o = o0; o < o1;) {
    const KOp* k = ops + o;
    const int type = k->type;
    if (type == KOP_GROUP) {
      // one 2x2 gate per register position: every matrix address comes from the
      // header, the four matrices are fetched together, then straight-line arithmetic
      const int4 h = *reinterpret_cast<const int4*>(k);
      const int s3 = k->nterms;
      const int s2 = k->cond;
      const float* m0 = kop_matrix(k + 1, h.z, variant);
      const float* m1 = kop_matrix(k + 2, h.w, variant);
      const float* m2 = kop_matrix(k + 3, s2, variant);
      const float* m3 = kop_matrix(k + 4, s3, variant);
      dense_reg<0>(a, m0);
      dense_reg<1>(a, m1);
      dense_reg<2>(a, m2);
      dense_reg<3>(a, m3);
      o += 1 + REG_BITS;
      continue;
    }
    ++o;
    const int cond = k->cond;
    if (cond >= 0 && !((blockbase >> cond) & 1)) continue;
    const float* m = kop_matrix(k, k->slot, variant);
    if (type == KOP_DENSE) {
      switch (k->a) {
        case 0: dense_reg<0>(a, m); break;
        case 1: dense_reg<1>(a, m); break;
        case 2: dense_reg<2>(a, m); break;
        default: dense_reg<3>(a, m); break;
      }
    } else if (type == KOP_DIAG) {
      const int j = k->a;
      const float2 d0 = make_float2(m[0], m[1]), d1 = make_float2(m[6], m[7]);
#pragma unroll
      for (int e = 0; e < R; ++e) a[e] = cmul(((idx[e] >> j) & 1) ? d1 : d0, a[e]);
    } else if (type == KOP_CZL) {
      const uint32_t* t = reinterpret_cast<const uint32_t*>(k->m);
      const int nt = k->nterms;
#pragma unroll
      for (int e = 0; e < R; ++e) {
        const uint32_t i = (uint32_t)idx[e];
        uint32_t par = 0;
        for (int q = 0; q < nt; ++q) par ^= __popc(i & (i >> t[2 * q]) & t[2 * q + 1]);
        if (par & 1) a[e] = make_float2(-a[e].x, -a[e].y);
      }
    } else if (type == KOP_SCALAR) {
      const bool bit = (blockbase >> k->a) & 1;
      const float2 ph = bit ? make_float2(m[6], m[7]) : make_float2(m[0], m[1]);
#pragma unroll
      for (int e = 0; e < R; ++e) a[e] = cmul(ph, a[e]);
    } else {  // KOP_CXL: control local bit a, target register position b
      switch (k->b) {
        case 0: cx_reg<0>(a, idx, k->a); break;
        case 1: cx_reg<1>(a, idx, k->a); break;
        case 2: cx_reg<2>(a, idx, k->a); break;
        default: cx_reg<3>(a, idx, k->a); break;
      }
    }
  }
}

// Ops one at a time over the whole LDS block (small blocks).
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

template <int NT>
__global__ __launch_bounds__(NT) void k_sim(const SimJob* __restrict__ jobs, int n_jobs, int total_wg,
                                            int wg_offset, const PassDesc* __restrict__ passes,
                                            const StageDesc* __restrict__ stages, const KOp* __restrict__ ops,
                                            float2* __restrict__ base) {
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
      if (tid == 0 && blockbase == 0) sh[0] = make_float2(1.f, 0.f);
    } else {
      for (int i = tid; i < nb; i += NT) sh[pad(i)] = st[blockbase + lo_tab[i & (TAB - 1)] + hi_tab[i >> 7]];
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
          run_stage_ops(a, idx, ops, S->op_begin, S->op_begin + S->op_count, blockbase, job.variant);
#pragma unroll
          for (int e = 0; e < R; ++e) sh[pb + S->proff[e]] = a[e];
        }
        __syncthreads();
      }
    }

    for (int i = tid; i < nb; i += NT) st[blockbase + lo_tab[i & (TAB - 1)] + hi_tab[i >> 7]] = sh[pad(i)];
    __syncthreads();
  }
}

constexpr size_t shmem_bytes(int bmax) {
  return 2 * TAB * sizeof(uint64_t) + sizeof(float2) * (((size_t)1 << bmax) + ((size_t)1 << bmax) / 16);
}

template <int NT>
int launch_sim_t(const SimJob* d_jobs, int n_jobs, int total_wg, int wg_offset, const PassDesc* d_passes,
                 const StageDesc* d_stages, const KOp* d_ops, float* base, int bmax, int grid, hipStream_t s) {
  const size_t shmem = shmem_bytes(bmax);
  static bool attr_set = false;
  if (!attr_set) {
    CCUT_HIP(hipFuncSetAttribute((const void*)k_sim<NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)shmem_bytes(PASS_MAX_B)));
    attr_set = true;
  }
  ProfScope prof(PROF_SIM, s);
  hipLaunchKernelGGL(k_sim<NT>, dim3(grid), dim3(NT), shmem, s, d_jobs, n_jobs, total_wg, wg_offset, d_passes,
                     d_stages, d_ops, reinterpret_cast<float2*>(base));
  CCUT_HIP(hipGetLastError());
  return 0;
}

}  // namespace

int launch_sim(const SimJob* d_jobs, int n_jobs, int total_wg, int wg_offset, const PassDesc* d_passes,
               const StageDesc* d_stages, const KOp* d_ops, float* base, int bmax, int threads, int grid_cap,
               hipStream_t s) {
  if (total_wg <= 0 || n_jobs <= 0) return 0;
  if (bmax < 1 || bmax > PASS_MAX_B) return fail(CCUT_EINVAL, "bad block bits %d", bmax);
  const int grid = (grid_cap > 0 && grid_cap < total_wg) ? grid_cap : total_wg;
  switch (threads) {
    case 256:
      return launch_sim_t<256>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_stages, d_ops, base, bmax, grid, s);
    case 512:
      return launch_sim_t<512>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_stages, d_ops, base, bmax, grid, s);
    case 1024:
      return launch_sim_t<1024>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_stages, d_ops, base, bmax, grid, s);
    default:
      return fail(CCUT_EINVAL, "unsupported workgroup size %d", threads);
  }
}

}  // namespace ccut
