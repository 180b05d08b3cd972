// LDS layout of the split-precision paired-column levels (fft_mfma.hip),
// shared with the planner that sizes their launches.
#pragma once

#include "fft_internal.h"

namespace moa {

// LDS elements after the scale slots of a paired matrix-core level: the
// stage-1 twiddles of every operand slot of a wave (64 lanes x 4).
constexpr int kMfmaPairTwElems = 256;

// These levels add a spare slot after every 256 elements to the one after
// every 16: their last radix-16 stage of a 4096-point column has the 16
// lanes of one LDS cycle write the 16 outputs of one butterfly, 256
// elements apart -- one bank pair under the 16-element padding alone.
__host__ __device__ constexpr inline int mfma_lds_pad(int i) { return i + (i >> 4) + (i >> 8); }
__host__ __device__ constexpr inline int mfma_lds_padded_len(int n) { return mfma_lds_pad(n - 1) + 1; }

// Column stride of such a tile: the rounding of lds_col_stride applied to
// the longer padded column.
__host__ __device__ constexpr inline int mfma_lds_col_stride(int n, int lanes_per_col)
{
    const int base = mfma_lds_padded_len(n);
    const int want = lanes_per_col >= 16 ? 0 : (lanes_per_col <= 0 ? 1 : lanes_per_col);
    return want == 0 ? base : base + ((want - (base & 31) + 32) & 31);
}

}  // namespace moa
