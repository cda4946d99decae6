// Band-limit changes of the truncated solves (Sect. 3: the transforms of a sweep
// stop at l_max^SHT = l_iter + margin while lambda is large). A packed alm array of
// band limit ls is copied into the packed layout of band limit ld >= ls, with the
// modes l > ls set to zero.
#include <hip/hip_runtime.h>

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

}  // namespace

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
