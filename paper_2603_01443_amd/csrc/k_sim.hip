// State-vector simulation kernel for gfx950 (Algorithm 2 of the paper, and
// the uncut baseline T_orig of Sec. III.A).
//
// A workgroup owns a block of 2^b amplitudes of one state: the amplitudes whose
// register qubits outside the pass group are fixed to the bits of the block id.
// The block is loaded into LDS (or generated as |0...0> on the first pass),
// every op of the pass is applied in LDS, and the block is written back once.
// When a state has at most 2^14 amplitudes the whole state is one block, so a
// subcircuit variant is simulated start to finish on chip and its final state
// is the only HBM traffic.  The low register qubits always belong to the
// group, so global loads and stores run over contiguous amplitude ranges.
//
// One launch covers a list of jobs (state, pass, variant); a grid-stride loop
// over the job list makes the launch persistent when the grid is smaller than
// the work.
#include "ccut_internal.h"

namespace ccut {

namespace {

constexpr int TAB = 128;  // offset-table entries per half (local bits 0..6 / 7..13)

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ float2 cmadd2(float2 m0, float2 x, float2 m1, float2 y) {
  return make_float2(m0.x * x.x - m0.y * x.y + m1.x * y.x - m1.y * y.y,
                     m0.x * x.y + m0.y * x.x + m1.x * y.y + m1.y * y.x);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_sim(const SimJob* __restrict__ jobs, int n_jobs, int total_wg,
                                            int wg_offset, const PassDesc* __restrict__ passes,
                                            const KOp* __restrict__ ops, float2* __restrict__ base) {
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
      for (int i = tid; i < nb; i += NT) sh[i] = make_float2(0.f, 0.f);
      __syncthreads();
      if (tid == 0 && blockbase == 0) sh[0] = make_float2(1.f, 0.f);
    } else {
      for (int i = tid; i < nb; i += NT) sh[i] = st[blockbase + lo_tab[i & (TAB - 1)] + hi_tab[i >> 7]];
    }
    __syncthreads();

    const int op_end = P->op_begin + P->op_count;
    for (int o = P->op_begin; o < op_end; ++o) {
      const KOp* k = ops + o;
      const int cond = k->cond;
      if (cond >= 0 && !((blockbase >> cond) & 1)) continue;
      const int slot = k->slot;
      const float* m = k->m + ((slot >= 0) ? 8 * ((job.variant >> slot) & 1) : 0);
      const int type = k->type;
      if (type == KOP_DENSE) {
        const int j = k->a;
        const float2 m00 = make_float2(m[0], m[1]), m01 = make_float2(m[2], m[3]);
        const float2 m10 = make_float2(m[4], m[5]), m11 = make_float2(m[6], m[7]);
        const int low = (1 << j) - 1;
        for (int p = tid; p < (nb >> 1); p += NT) {
          const int i0 = ((p & ~low) << 1) | (p & low);
          const int i1 = i0 | (1 << j);
          const float2 x = sh[i0], y = sh[i1];
          sh[i0] = cmadd2(m00, x, m01, y);
          sh[i1] = cmadd2(m10, x, m11, y);
        }
      } else if (type == KOP_DIAG) {
        const int j = k->a;
        const float2 d0 = make_float2(m[0], m[1]), d1 = make_float2(m[6], m[7]);
        const bool one0 = (m[0] == 1.f && m[1] == 0.f);
        const int low = (1 << j) - 1;
        for (int p = tid; p < (nb >> 1); p += NT) {
          const int i0 = ((p & ~low) << 1) | (p & low);
          const int i1 = i0 | (1 << j);
          if (!one0) sh[i0] = cmul(d0, sh[i0]);
          sh[i1] = cmul(d1, sh[i1]);
        }
      } else if (type == KOP_CZL) {
        const uint32_t* t = reinterpret_cast<const uint32_t*>(k->m);
        const int nt = k->nterms;
        for (int i = tid; i < nb; i += NT) {
          uint32_t par = 0;
          for (int q = 0; q < nt; ++q) par ^= __popc((uint32_t)i & ((uint32_t)i >> t[2 * q]) & t[2 * q + 1]);
          if (par & 1) {
            float2 v = sh[i];
            sh[i] = make_float2(-v.x, -v.y);
          }
        }
      } else if (type == KOP_SCALAR) {
        const bool bit = (blockbase >> k->a) & 1;
        const float2 ph = bit ? make_float2(m[6], m[7]) : make_float2(m[0], m[1]);
        if (!(ph.x == 1.f && ph.y == 0.f))
          for (int i = tid; i < nb; i += NT) sh[i] = cmul(ph, sh[i]);
      } else {  // KOP_CXL
        const int c = k->a, j = k->b;
        const int low = (1 << j) - 1;
        for (int p = tid; p < (nb >> 1); p += NT) {
          const int i0 = ((p & ~low) << 1) | (p & low);
          if ((i0 >> c) & 1) {
            const int i1 = i0 | (1 << j);
            const float2 x = sh[i0];
            sh[i0] = sh[i1];
            sh[i1] = x;
          }
        }
      }
      __syncthreads();
    }

    for (int i = tid; i < nb; i += NT) st[blockbase + lo_tab[i & (TAB - 1)] + hi_tab[i >> 7]] = sh[i];
    __syncthreads();
  }
}

template <int NT>
int launch_sim_t(const SimJob* d_jobs, int n_jobs, int total_wg, int wg_offset, const PassDesc* d_passes,
                 const KOp* d_ops, float* base, int bmax, int grid, hipStream_t s) {
  const size_t shmem = 2 * TAB * sizeof(uint64_t) + (sizeof(float2) << bmax);
  static bool attr_set = false;
  if (!attr_set) {
    CCUT_HIP(hipFuncSetAttribute((const void*)k_sim<NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)(2 * TAB * sizeof(uint64_t) + (sizeof(float2) << PASS_MAX_B))));
    attr_set = true;
  }
  ProfScope prof(PROF_SIM, s);
  hipLaunchKernelGGL(k_sim<NT>, dim3(grid), dim3(NT), shmem, s, d_jobs, n_jobs, total_wg, wg_offset, d_passes,
                     d_ops, reinterpret_cast<float2*>(base));
  CCUT_HIP(hipGetLastError());
  return 0;
}

}  // namespace

int launch_sim(const SimJob* d_jobs, int n_jobs, int total_wg, int wg_offset, const PassDesc* d_passes,
               const KOp* d_ops, float* base, int bmax, int threads, int grid_cap, hipStream_t s) {
  if (total_wg <= 0 || n_jobs <= 0) return 0;
  if (bmax < 1 || bmax > PASS_MAX_B) return fail(CCUT_EINVAL, "bad block bits %d", bmax);
  const int grid = (grid_cap > 0 && grid_cap < total_wg) ? grid_cap : total_wg;
  switch (threads) {
    case 256: return launch_sim_t<256>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_ops, base, bmax, grid, s);
    case 512: return launch_sim_t<512>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_ops, base, bmax, grid, s);
    case 1024: return launch_sim_t<1024>(d_jobs, n_jobs, total_wg, wg_offset, d_passes, d_ops, base, bmax, grid, s);
    default: return fail(CCUT_EINVAL, "unsupported workgroup size %d", threads);
  }
}

}  // namespace ccut
