// Reduce-scatter butterfly over one 64-lane wave, shared by the Gram-Schmidt
// passes and the reduction fused into the DG tangent kernel.
#pragma once

#include <hip/hip_runtime.h>

namespace pcexp {

// Step (H, O) halves the values a lane holds, sending H of them to lane ^ O
// and adding the H it receives.  Run as Bfly<NP / 2, 32> on NP (a power of
// two, <= 64) values per lane: afterwards a[0] holds the wave's sum of column
// `col`, on every lane of each group of 64 / NP consecutive lanes.  NP - 1 +
// log2(64 / NP) shuffles in all, instead of 6 per column.  All indices are
// compile-time constants.
template <int H, int O>
struct Bfly {
  static __device__ __forceinline__ void run(double* a, int lane, int& col) {
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double send = up ? a[i] : a[i + H];
      const double keep = up ? a[i + H] : a[i];
      a[i] = keep + __shfl_xor(send, O, 64);
    }
    if (up) col += H;
    Bfly<H / 2, O / 2>::run(a, lane, col);
  }
};
template <int O> struct Bfly<0, O> {          // fewer columns than lanes: finish with plain shuffles
  static __device__ __forceinline__ void run(double* a, int, int&) {
#pragma unroll
    for (int o = O; o >= 1; o /= 2) a[0] += __shfl_xor(a[0], o, 64);
  }
};
template <int H> struct Bfly<H, 0> {
  static __device__ __forceinline__ void run(double*, int, int&) {}
};
template <> struct Bfly<0, 0> {
  static __device__ __forceinline__ void run(double*, int, int&) {}
};

}  // namespace pcexp
