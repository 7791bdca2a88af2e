// Kernel launch helper.  Every launch of the library goes through launch();
// when the profiling hook has armed an event pair, the pair is handed to the
// dispatch itself (hipExtLaunchKernel), so the events carry the kernel's own
// start and end timestamps rather than those of markers around it.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace pcexp {

struct LaunchTiming {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
// Armed by the profiling hook for the next launch on this host thread.
extern thread_local LaunchTiming g_launch_timing;

template <typename F, typename... Args>
inline void launch(F kernel, const dim3& grid, const dim3& block, unsigned shmem, hipStream_t st, Args... args) {
  LaunchTiming& t = g_launch_timing;
  hipEvent_t a = t.start, b = t.stop;
  t.start = t.stop = nullptr;
  hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, a, b, 0u, args...);
}

}  // namespace pcexp
