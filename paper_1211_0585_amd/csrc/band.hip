// Small device utilities of the host runtime.
//
// Band-limit changes of the truncated solves (Sect. 3: the transforms of a sweep
// stop at l_max^SHT = l_iter + margin while lambda is large): a packed alm array of
// band limit ls is copied into the packed layout of band limit ld >= ls, with the
// modes l > ls set to zero.
//
// Zero fills by a kernel rather than hipMemsetAsync, so that a caller may record
// the work in a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace mwf {

namespace {

// One workgroup per m (0 <= m <= ld); entry (l, m) of band limit L sits at
// m (2 L + 1 - m) / 2 + l. Reads stay below the source's (ls+1)(ls+2)/2 entries:
// they happen only for m <= l <= ls.
template <class T2>
__global__ void alm_repack_kernel(const T2* __restrict__ src, int ls, T2* __restrict__ dst, int ld) {
  const int m = blockIdx.x;
  const int64_t doff = (int64_t)m * (2 * ld + 1 - m) / 2;
  const int64_t soff = (int64_t)m * (2 * ls + 1 - m) / 2;
  for (int l = m + (int)threadIdx.x; l <= ld; l += (int)blockDim.x) {
    T2 v;
    v.x = 0;
    v.y = 0;
    if (l <= ls) v = src[soff + l];
    dst[doff + l] = v;
  }
}

__global__ void zero_fill_kernel(uint4* __restrict__ p, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

}  // namespace

hipError_t launch_zero_fill(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (!p || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(p) % 16 != 0) return hipErrorInvalidValue;
  const size_t n16 = bytes / 16;
  const unsigned blocks = (unsigned)std::min<size_t>(1024, (n16 + 255) / 256);
  hipLaunchKernelGGL(zero_fill_kernel, dim3(blocks), dim3(256), 0, s, static_cast<uint4*>(p), n16);
  return hipGetLastError();
}

hipError_t launch_alm_repack(const void* src, int ls, void* dst, int ld, bool fp64, hipStream_t s) {
  if (ls < 0 || ld < ls || !src || !dst) return hipErrorInvalidValue;
  if (fp64)
    hipLaunchKernelGGL(alm_repack_kernel<double2>, dim3(ld + 1), dim3(256), 0, s, static_cast<const double2*>(src),
                       ls, static_cast<double2*>(dst), ld);
  else
    hipLaunchKernelGGL(alm_repack_kernel<float2>, dim3(ld + 1), dim3(256), 0, s, static_cast<const float2*>(src), ls,
                       static_cast<float2*>(dst), ld);
  return hipGetLastError();
}

}  // namespace mwf
