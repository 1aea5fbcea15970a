// Split-precision MFMA merge: launch interface.
#pragma once

#include "ccut_internal.h"

namespace ccut {

enum MergeMfmaMode : int { MERGE_BF16X3 = 1, MERGE_FP16X3 = 2, MERGE_BF16 = 3, MERGE_FP16X2 = 4 };

struct MergeMfmaArgs {
  const float2* A;          // low-qubit factor (K terms of 2^qx), weights applied
  uint64_t a_kstride, a_bstride;
  const float2* B;          // high-qubit factor (K terms of 2^qy)
  uint64_t b_kstride, b_bstride;
  const float2* w;          // K complex weights
  int K, qx, qy, S;         // S = ceil(2K / 16) MFMA steps
  int batch, r_batch;       // output batch; R planes per batch (1 when the A side is shared)
  uint4 *Lhi, *Llo, *Rhi, *Rlo;
  uint64_t l_plane_stride, r_plane_stride;  // uint4 elements per batch entry
  float* out;
  uint64_t out_bstride;     // complex64 elements
};

bool merge_mfma_supported(int qx, int qy);
// variant 0..3, bit 0: stores through an LDS transpose (else direct accumulator stores);
//               bit 1: 64-row tiles, 32 rows per wavefront (else 128-row tiles);
// variant 4: R-stationary kernel (a 128-column strip of R held in LDS by one
//            16-wavefront workgroup per CU), up to 8 MFMA steps (K <= 64); above
//            that it runs as variant 1.
// variant 5: LDS-staged kernel for many steps: one 8-wavefront workgroup per CU
//            over 256 x 256 tiles, each step's fragments copied from L2 straight
//            into LDS once per tile (four buffers); needs qy >= 8 and K >= 32,
//            else it runs as variant 1.
// variant 6: column-stationary kernel: one 8-wavefront workgroup per CU and
//            256-column strip; four wavefronts hold two column blocks' R fragments
//            each in registers and compute, four fetch the row blocks' L fragments
//            into LDS and store each 32 x 256 tile through LDS as whole 1 KiB row
//            segments; K <= 64 (else variant 1).
// grid_cap > 0: persistent grid of at most grid_cap workgroups per batch entry.
int launch_merge_mfma(const MergeMfmaArgs& a, int mode, int variant, int grid_cap, hipStream_t s);

// uint4 elements of one L (rows) / R (columns) plane for a stage
inline uint64_t mfma_l_plane(int qy, int S) { return ((uint64_t)1 << qy) / 32 * S * 64; }
inline uint64_t mfma_r_plane(int qx, int S) { return ((uint64_t)2 << qx) / 32 * S * 64; }
inline int mfma_steps(int K) { return (2 * K + 15) / 16; }

}  // namespace ccut
