// The non-edge table of ltab.h as the kernels stage it in LDS (device code).
#pragma once

#include <hip/hip_runtime.h>

#include "ltab.h"
#include "pairfn.h"

namespace gempe {

constexpr int kLtabF4 = GEMPE_LTAB_SEGS + 1;                           // the segments and the all-zero one past them
constexpr int kLtabZero = (int)(-GEMPE_LTAB_LO * GEMPE_LTAB_INV_H);    // the segment of tau = 0
constexpr unsigned kLtabSegs = GEMPE_LTAB_SEGS;

// Copies the one-gather table (kLtabF4 float4) into LDS in the form pair_nonedge_tab reads,
// c0 raised by kTabLogScale, with the threads of the workgroup; the caller's barrier orders
// the copy before any use.
__device__ __forceinline__ void stage_ltab(float4 *dst) {
    const float4 *src = reinterpret_cast<const float4 *>(kLtab);
    for (int q = threadIdx.x; q < kLtabF4; q += blockDim.x) {
        float4 e = src[q];
        e.x += kTabLogScale;
        dst[q] = e;
    }
}

}  // namespace gempe
