// Dynamic item distribution for persistent launches.
#pragma once

#include <hip/hip_runtime.h>

#include "blfls_internal.h"

namespace blfls {

// Next item of this workgroup, >= total when the work is exhausted.  With
// per_xcd, the items are split into 8 contiguous ranges, one per XCD (workgroup
// b runs on XCD b mod 8), and each range has its own counter.
__device__ __forceinline__ int grab_item(int* counters, int total, bool per_xcd) {
  __shared__ int s_item;
  if (threadIdx.x == 0) {
    int item;
    if (per_xcd) {
      const int x = static_cast<int>(blockIdx.x % kXcds);
      const int q = total / kXcds, rem = total % kXcds;
      const int start = x * q + min(x, rem);
      const int count = q + (x < rem ? 1 : 0);
      const int c = atomicAdd(&counters[x], 1);
      item = c < count ? start + c : total;
    } else {
      item = atomicAdd(&counters[0], 1);
    }
    s_item = item;
  }
  __syncthreads();
  const int item = s_item;
  __syncthreads();  // every thread has read s_item before it is overwritten
  return item;
}

}  // namespace blfls
