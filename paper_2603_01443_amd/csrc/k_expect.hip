// Expectation values of Pauli strings without the O(2^q) merge (the setting
// the paper names as its next step, Sec. VI).
//
// For O = P_{n-1} x ... x P_0 (one Pauli string per segment) and the cut
// state Psi = sum_b alpha_b (x)_i psi_i^{(r_i(b))}:
//   <Psi|O|Psi> = sum_{b,b'} conj(alpha_b) alpha_b' prod_i G_i[r_i(b)][r_i(b')],
//   G_i[r][r'] = <psi_i^{(r)}| P_i |psi_i^{(r')}>.
// k_gram forms the V x V matrix G_i (V = 2^{c_i}) of one segment: a complex
// product of two V x N operands (the states, and the states with P_i applied)
// contracted over the N = 2^{q_i} amplitudes.  P_i acts as an index flip (X, Y)
// and a sign (Z, Y) while the right-hand chunk is staged; the constant
// (-i)^{#Y} is applied by the host.
//
// Tiling: a workgroup owns a TM x TM tile of G and a range of amplitudes
// (grid.y splits the range so that small V still fills the device).  Chunks
// of CH amplitudes of the TM left and TM right rows are staged in LDS
// (amplitude-major, so the 16 threads of a tile row read 16 consecutive
// columns); each of the 256 threads accumulates a (TM/16) x (TM/16) block of
// entries, rows ty + 16 i and columns tx + 16 j.  Products are float32 (the
// states are complex64), summed per chunk in float32 and across chunks in
// float64.  Each split writes its own partial tile; k_gram_sum adds the
// partials in split order, so the result does not depend on scheduling.
#include "ccut_internal.h"

namespace ccut {

namespace {

constexpr int CH = 32;  // amplitudes per staged chunk

template <int TM>
__global__ __launch_bounds__(256) void k_gram(const float2* __restrict__ states, int V, uint64_t N,
                                              uint32_t flip, uint32_t zy, uint64_t per_split,
                                              double2* __restrict__ part) {
  constexpr int R = TM / 16;  // entries per thread along each side
  __shared__ float2 As[CH][TM + 1], Bs[CH][TM + 1];
  const int tiles_side = V > TM ? V / TM : 1;
  const int tr = (int)blockIdx.x / tiles_side, tc = (int)blockIdx.x % tiles_side;
  const int t = threadIdx.x, ty = t / 16, tx = t % 16;
  const uint64_t x_begin = (uint64_t)blockIdx.y * per_split;
  const uint64_t x_end = x_begin + per_split < N ? x_begin + per_split : N;
  double accr[R][R], acci[R][R];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) accr[i][j] = acci[i][j] = 0.0;
  for (uint64_t x0 = x_begin; x0 < x_end; x0 += CH) {
    // stage: element e = (row, col) with col fastest, so a wavefront reads
    // 2 rows x 32 consecutive amplitudes (256-byte runs; the flip keeps runs
    // contiguous up to a permutation inside the chunk)
#pragma unroll
    for (int e = t; e < TM * CH; e += 256) {
      const int row = e / CH, col = e % CH;
      const uint64_t x = x0 + col;
      const int ra = tr * TM + row, rb = tc * TM + row;
      float2 a = make_float2(0.f, 0.f), b = make_float2(0.f, 0.f);
      if (x < x_end) {
        if (ra < V) a = states[(uint64_t)ra * N + x];
        if (rb < V) {
          b = states[(uint64_t)rb * N + (x ^ flip)];
          if (__popcll(x & zy) & 1) b = make_float2(-b.x, -b.y);
        }
      }
      As[col][row] = a;
      Bs[col][row] = b;
    }
    __syncthreads();
    float sr[R][R], si[R][R];
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int j = 0; j < R; ++j) sr[i][j] = si[i][j] = 0.f;
#pragma unroll 4
    for (int xx = 0; xx < CH; ++xx) {
      float2 a[R], b[R];
#pragma unroll
      for (int i = 0; i < R; ++i) a[i] = As[xx][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < R; ++j) b[j] = Bs[xx][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
          sr[i][j] += a[i].x * b[j].x + a[i].y * b[j].y;  // conj(a) * b
          si[i][j] += a[i].x * b[j].y - a[i].y * b[j].x;
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int j = 0; j < R; ++j) {
        accr[i][j] += sr[i][j];
        acci[i][j] += si[i][j];
      }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int r = tr * TM + ty + 16 * i, rp = tc * TM + tx + 16 * j;
      if (r < V && rp < V) part[((uint64_t)blockIdx.y * V + r) * V + rp] = make_double2(accr[i][j], acci[i][j]);
    }
}

// out[e] = sum over splits s (in order) of part[s][e], e < V * V
__global__ __launch_bounds__(256) void k_gram_sum(const double2* __restrict__ part, uint64_t VV, int splits,
                                                  double2* __restrict__ out) {
  const uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= VV) return;
  double re = 0.0, im = 0.0;
  for (int s = 0; s < splits; ++s) {
    const double2 p = part[(uint64_t)s * VV + e];
    re += p.x;
    im += p.y;
  }
  out[e] = make_double2(re, im);
}

}  // namespace

// Tile side and number of amplitude-range splits for a V x V matrix over N
// amplitudes: the largest tile (fewest LDS reads per product) that still gives
// a workgroup per compute unit, with about 512 workgroups in all and at least 4
// chunks per workgroup (the partial tiles stay small next to the states read).
GramShape gram_shape(int V, uint64_t N) {
  const uint64_t chunks = (N + CH - 1) / CH;
  GramShape g{16, 1};
  for (int tm = 64; tm >= 16; tm /= 2) {
    if (tm > 16 && tm > V) continue;
    const uint64_t side = V > tm ? (uint64_t)(V / tm) : 1;
    const uint64_t tiles = side * side;
    uint64_t sp = tiles >= 512 ? 1 : (512 + tiles - 1) / tiles;
    if (sp > chunks / 4) sp = chunks / 4;
    if (sp < 1) sp = 1;
    g = GramShape{tm, (int)sp};
    if (tiles * sp >= 256) break;
  }
  return g;
}

int launch_gram(const float2* states, int V, uint64_t N, uint32_t flip, uint32_t zy, GramShape g, double2* part,
                double2* out, hipStream_t s) {
  const int TM = g.tm;
  const int side = V > TM ? V / TM : 1;
  const uint64_t chunks = (N + CH - 1) / CH;
  const uint64_t per = ((chunks + g.splits - 1) / g.splits) * CH;
  const dim3 grid((unsigned)(side * side), (unsigned)g.splits);
  ProfScope prof(PROF_EXPECT, s);
  if (TM == 64)
    hipLaunchKernelGGL(k_gram<64>, grid, dim3(256), 0, s, states, V, N, flip, zy, per, part);
  else if (TM == 32)
    hipLaunchKernelGGL(k_gram<32>, grid, dim3(256), 0, s, states, V, N, flip, zy, per, part);
  else
    hipLaunchKernelGGL(k_gram<16>, grid, dim3(256), 0, s, states, V, N, flip, zy, per, part);
  CCUT_HIP(hipGetLastError());
  const uint64_t VV = (uint64_t)V * V;
  hipLaunchKernelGGL(k_gram_sum, dim3((unsigned)((VV + 255) / 256)), dim3(256), 0, s, part, VV, g.splits, out);
  CCUT_HIP(hipGetLastError());
  return 0;
}

}  // namespace ccut
