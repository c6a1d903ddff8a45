// Bandwidth calibration: the memory streams of one fused step (57 planes
// read: 19 populations, 10 history, 28 geometry; 29 planes written: 19
// populations, 10 history) with none of its arithmetic, one node per thread,
// streaming loads and stores.  Its time is the practical floor of a step on
// this layout, beside the 8 TB/s peak.
#include "lbm_internal.h"

namespace lbm {

namespace {

constexpr int PR = 19 + H_N + G_N, PW = 19 + H_N;

template <class T>
__global__ __launch_bounds__(256) void k_stream_probe(const T* __restrict__ in, T* __restrict__ out, unsigned n) {
  const unsigned i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  T s = T(0);
#pragma unroll
  for (int p = 0; p < PR; ++p) s += __builtin_nontemporal_load(in + (size_t)p * n + i);
#pragma unroll
  for (int q = 0; q < PW; ++q) __builtin_nontemporal_store(s + T(q), out + (size_t)q * n + i);
}

}  // namespace

hipError_t launch_stream_probe(int precision, long long n, const void* in, void* out, hipStream_t s) {
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (precision == 0)
    hipLaunchKernelGGL(k_stream_probe<double>, dim3(grid), dim3(256), 0, s, (const double*)in, (double*)out,
                       (unsigned)n);
  else
    hipLaunchKernelGGL(k_stream_probe<float>, dim3(grid), dim3(256), 0, s, (const float*)in, (float*)out,
                       (unsigned)n);
  return hipGetLastError();
}

}  // namespace lbm
