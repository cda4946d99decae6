// Constrained realisations (Sect. 3: Wiener-filter map plus fluctuation map): the
// signal draw's alm from unit draws, the data map of the modified solve, and the
// final sums. The random numbers are the caller's; arithmetic is FP64, stored in
// the plan's type.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace mwf {

namespace {

template <class T>
struct Cplx;
template <>
struct Cplx<double> {
  using type = double2;
};
template <>
struct Cplx<float> {
  using type = float2;
};

// out = sqrt(C_l) xi (accumulate: out += sqrt(C_l) xi) over the packed alm; one
// workgroup per (m, map), entries (l, m) at m (2 lmax + 1 - m) / 2 + l. The draw's
// imaginary part at m = 0 is dropped (real field).
template <class T>
__global__ void cr_alm_kernel(const double* __restrict__ cl, int lmax, int64_t nalm,
                              const typename Cplx<T>::type* __restrict__ xi, typename Cplx<T>::type* out,
                              int accumulate) {
  const int m = blockIdx.x;
  const int64_t base = (int64_t)blockIdx.y * nalm + (int64_t)m * (2 * lmax + 1 - m) / 2;
  for (int l = m + (int)threadIdx.x; l <= lmax; l += (int)blockDim.x) {
    const double c = sqrt(cl[l]);
    const typename Cplx<T>::type x = xi[base + l];
    double re = c * (double)x.x;
    double im = m == 0 ? 0.0 : c * (double)x.y;
    if (accumulate) {
      re += (double)out[base + l].x;
      im += (double)out[base + l].y;
    }
    typename Cplx<T>::type v;
    v.x = (T)re;
    v.y = (T)im;
    out[base + l] = v;
  }
}

// out = d - s_rand - n_rand with n_rand = eta sqrt(tau / q) (q = tau ninv; 0 where q = 0).
template <class T>
__global__ void cr_data_kernel(const T* __restrict__ d, const T* __restrict__ srand, const T* __restrict__ eta,
                               const T* __restrict__ q, double tau, T* __restrict__ out, int64_t npix,
                               int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const double qp = (double)q[i % npix];
    const double n = qp > 0.0 ? (double)eta[i] * sqrt(tau / qp) : 0.0;
    out[i] = (T)((double)d[i] - (double)srand[i] - n);
  }
}

// out += s_rand
template <class T>
__global__ void cr_add_kernel(T* __restrict__ out, const T* __restrict__ srand, int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (T)((double)out[i] + (double)srand[i]);
}

dim3 flat_grid(int64_t total) { return dim3((unsigned)std::min<int64_t>((total + 255) / 256, 8192)); }

}  // namespace

hipError_t launch_cr_alm(const double* cl, int lmax, int64_t nalm, int nmaps, const void* xi, void* out,
                         bool accumulate, bool fp64, hipStream_t s) {
  if (lmax < 0 || nmaps < 1) return hipErrorInvalidValue;
  const dim3 grid(lmax + 1, nmaps);
  if (fp64)
    hipLaunchKernelGGL(cr_alm_kernel<double>, grid, dim3(256), 0, s, cl, lmax, nalm, static_cast<const double2*>(xi),
                       static_cast<double2*>(out), accumulate ? 1 : 0);
  else
    hipLaunchKernelGGL(cr_alm_kernel<float>, grid, dim3(256), 0, s, cl, lmax, nalm, static_cast<const float2*>(xi),
                       static_cast<float2*>(out), accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_cr_data(const void* d, const void* srand, const void* eta, const void* q, double tau, void* out,
                          int64_t npix, int nmaps, bool fp64, hipStream_t s) {
  const int64_t total = npix * nmaps;
  if (total < 1) return hipErrorInvalidValue;
  if (fp64)
    hipLaunchKernelGGL(cr_data_kernel<double>, flat_grid(total), dim3(256), 0, s, static_cast<const double*>(d),
                       static_cast<const double*>(srand), static_cast<const double*>(eta),
                       static_cast<const double*>(q), tau, static_cast<double*>(out), npix, total);
  else
    hipLaunchKernelGGL(cr_data_kernel<float>, flat_grid(total), dim3(256), 0, s, static_cast<const float*>(d),
                       static_cast<const float*>(srand), static_cast<const float*>(eta), static_cast<const float*>(q),
                       tau, static_cast<float*>(out), npix, total);
  return hipGetLastError();
}

hipError_t launch_cr_add(void* out, const void* srand, int64_t total, bool fp64, hipStream_t s) {
  if (total < 1) return hipErrorInvalidValue;
  if (fp64)
    hipLaunchKernelGGL(cr_add_kernel<double>, flat_grid(total), dim3(256), 0, s, static_cast<double*>(out),
                       static_cast<const double*>(srand), total);
  else
    hipLaunchKernelGGL(cr_add_kernel<float>, flat_grid(total), dim3(256), 0, s, static_cast<float*>(out),
                       static_cast<const float*>(srand), total);
  return hipGetLastError();
}

}  // namespace mwf
