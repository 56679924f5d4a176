// Host emulation: the dispatch-recorded events of hipExtLaunchKernelGGL are
// not timed; the kernel runs as any other launch.
#pragma once
#include "hip_runtime.h"
template <typename... KArgs, typename... Args>
void hipExtLaunchKernelGGL(void (*k)(KArgs...), dim3 grid, dim3 block,
                           size_t shmem, hipStream_t s, hipEvent_t a,
                           hipEvent_t b, unsigned flags, Args... args) {
  (void)a;
  (void)b;
  (void)flags;
  hipLaunchKernelGGL(k, grid, block, shmem, s, args...);
}
