// Timeline record of one work item of a batched step: when the workgroup
// started and ended on the device's real-time clock, and which CU ran it.
#pragma once

#include <hip/hip_runtime.h>

namespace si {

// Record of workgroup blockIdx.x: {start, end, CU, item}; CU = XCC_ID << 16 |
// bits 15:8 of HW_ID (CU, shader array and engine within the XCC).  The
// workgroup synchronises first, so that `end` follows every wave's stores.
__device__ __forceinline__ void batch_trace_record(unsigned long long *trace,
                                                   unsigned long long start) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long end = wall_clock64();
    const unsigned hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);    // HW_ID
    const unsigned xcc = __builtin_amdgcn_s_getreg((31 << 11) | 20);  // XCC_ID
    unsigned long long *o = trace + (size_t)blockIdx.x * 4;
    o[0] = start;
    o[1] = end;
    o[2] = ((unsigned long long)(xcc & 0xFFFFu) << 16) | ((hw >> 8) & 0xFFu);
    o[3] = blockIdx.x;
  }
}

}  // namespace si
