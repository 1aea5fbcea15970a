// Expectation values of Pauli strings without the O(2^q) merge (the setting
// the paper names as its next step, Sec. VI).
//
// For O = P_{n-1} x ... x P_0 (one Pauli string per segment) and the cut
// state Psi = sum_b alpha_b (x)_i psi_i^{(r_i(b))}:
//   <Psi|O|Psi> = sum_{b,b'} conj(alpha_b) alpha_b' prod_i G_i[r_i(b)][r_i(b')],
//   G_i[r][r'] = <psi_i^{(r)}| P_i |psi_i^{(r')}>.
// This kernel forms the V x V matrix G_i (V = 2^{c_i}) of one segment as a
// tiled sum over the amplitudes: P_i acts as an index flip (X, Y) and a sign
// (Z, Y) on the right-hand state, the constant (-i)^{#Y} is applied by the
// host.  Products are float32 (the states are complex64), summed per 64
// amplitudes in float32 and across chunks in float64; the amplitude range is
// split over grid.y so that small V still spreads over the device, each split
// writing its own partial tile (summed in a fixed order by the host).
#include "ccut_internal.h"

namespace ccut {

namespace {

constexpr int ET = 16;  // tile side (entries of G)
constexpr int CH = 64;  // amplitudes per chunk

__global__ __launch_bounds__(256) void k_gram(const float2* __restrict__ states, int V, uint64_t N,
                                              uint32_t flip, uint32_t zy, uint64_t per_split,
                                              double2* __restrict__ part) {
  __shared__ float2 As[ET][CH + 1], Bs[ET][CH + 1];
  const int tiles_side = (V + ET - 1) / ET;
  const int tr = (int)blockIdx.x / tiles_side, tc = (int)blockIdx.x % tiles_side;
  const int t = threadIdx.x, ty = t / ET, tx = t % ET;
  const uint64_t x_begin = (uint64_t)blockIdx.y * per_split;
  const uint64_t x_end = x_begin + per_split < N ? x_begin + per_split : N;
  double accr = 0.0, acci = 0.0;
  for (uint64_t x0 = x_begin; x0 < x_end; x0 += CH) {
    for (int i = t; i < ET * CH; i += 256) {
      const int row = i / CH, col = i % CH;
      const uint64_t x = x0 + col;
      const int ra = tr * ET + row, rb = tc * ET + row;
      float2 a = make_float2(0.f, 0.f), b = make_float2(0.f, 0.f);
      if (x < x_end) {
        if (ra < V) a = states[(uint64_t)ra * N + x];
        if (rb < V) {
          b = states[(uint64_t)rb * N + (x ^ flip)];
          if (__popcll(x & zy) & 1) b = make_float2(-b.x, -b.y);
        }
      }
      As[row][col] = a;
      Bs[row][col] = b;
    }
    __syncthreads();
    float sr = 0.f, si = 0.f;
#pragma unroll 8
    for (int xx = 0; xx < CH; ++xx) {
      const float2 a = As[ty][xx], b = Bs[tx][xx];
      sr += a.x * b.x + a.y * b.y;  // conj(a) * b
      si += a.x * b.y - a.y * b.x;
    }
    accr += sr;
    acci += si;
    __syncthreads();
  }
  const int r = tr * ET + ty, rp = tc * ET + tx;
  if (r < V && rp < V) part[((uint64_t)blockIdx.y * V + r) * V + rp] = make_double2(accr, acci);
}

}  // namespace

// Splits of the amplitude range for a V x V matrix over N amplitudes (at least
// ~512 workgroups when the tiles alone give fewer).
int gram_splits(int V, uint64_t N) {
  const int tiles = ((V + ET - 1) / ET) * ((V + ET - 1) / ET);
  const uint64_t chunks = (N + CH - 1) / CH;
  uint64_t s = tiles >= 512 ? 1 : (512 + tiles - 1) / tiles;
  if (s > chunks) s = chunks;
  return s < 1 ? 1 : (int)s;
}

int launch_gram(const float2* states, int V, uint64_t N, uint32_t flip, uint32_t zy, int splits, double2* part,
                hipStream_t s) {
  const int tiles_side = (V + ET - 1) / ET;
  const uint64_t chunks = (N + CH - 1) / CH;
  const uint64_t per = ((chunks + splits - 1) / splits) * CH;
  ProfScope prof(PROF_EXPECT, s);
  hipLaunchKernelGGL(k_gram, dim3((unsigned)(tiles_side * tiles_side), (unsigned)splits), dim3(256), 0, s, states, V,
                     N, flip, zy, per, part);
  CCUT_HIP(hipGetLastError());
  return 0;
}

}  // namespace ccut
