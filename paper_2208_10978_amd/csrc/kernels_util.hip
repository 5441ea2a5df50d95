// Reductions and small utilities (FP64, fixed order, no atomics).
#include "device_common.h"
#include "launch.h"

namespace q2sv {

// Per block: partials[0][b] = sum Re(conj(a) b), partials[1][b] = sum |a|^2,
// partials[2][b] = sum d |a|^2 (the missing operands contribute zero).
template <typename T>
__global__ void __launch_bounds__(256) k_dot(const T* __restrict__ a, const T* __restrict__ b,
                                             const double* __restrict__ d, uint64_t n_amp,
                                             double* __restrict__ partials) {
  __shared__ double red[4];
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  double re = 0.0, nn = 0.0, dd = 0.0;
  for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < n_amp; i += stride) {
    const T u = a[i];
    const double p = (double)u.x * u.x + (double)u.y * u.y;
    nn += p;
    if (b) {
      const T v = b[i];
      re += (double)u.x * v.x + (double)u.y * v.y;
    }
    if (d) dd += d[i] * p;
  }
  const double s0 = block_sum<256>(re, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s0;
  const double s1 = block_sum<256>(nn, red);
  if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = s1;
  const double s2 = block_sum<256>(dd, red);
  if (threadIdx.x == 0) partials[2 * gridDim.x + blockIdx.x] = s2;
}

// partials[block] = how many of the block's amplitudes have a nonzero
// imaginary part (exact in FP64 below 2^53)
template <typename T>
__global__ void __launch_bounds__(256) k_imag_count(const T* __restrict__ a, uint64_t n_amp,
                                                    double* __restrict__ partials) {
  __shared__ double red[4];
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  double c = 0.0;
  for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < n_amp; i += stride) c += a[i].y != 0 ? 1.0 : 0.0;
  const double s = block_sum<256>(c, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// partials[block] = the largest binary exponent e with 2^(e-1) <= |re| + |im|
// over the block's amplitudes (kFxNone when all are zero), as a double: the
// fixed-point scale of a lambda build comes from their maximum.
template <typename T>
__global__ void __launch_bounds__(256) k_amp_exponent(const T* __restrict__ a, uint64_t n_amp,
                                                      double* __restrict__ partials) {
  __shared__ int red[4];
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  int e = kFxNone;
  for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < n_amp; i += stride)
    e = max(e, fx_exp(fabs((double)a[i].x) + fabs((double)a[i].y)));
  e = wave_max_i32(e);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = double(max(max(red[0], red[1]), max(red[2], red[3])));
}

// out[row] = sum_{j < len} in[row * stride + j], fixed order (one block per row)
__global__ void __launch_bounds__(256) k_reduce_rows(const double* __restrict__ in, uint64_t stride, uint32_t len,
                                                     double* __restrict__ out) {
  __shared__ double red[4];
  const uint64_t row = blockIdx.x;
  double s = 0.0;
  for (uint32_t j = threadIdx.x; j < len; j += 256) s += in[row * stride + j];
  const double t = block_sum<256>(s, red);
  if (threadIdx.x == 0) out[row] = t;
}

// out[0] = (sum_j sums[j]) / norm, out[1] = norm
__global__ void k_finish_energy(const double* __restrict__ sums, int nh, const double* __restrict__ norm,
                                double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double e = 0.0;
    for (int j = 0; j < nh; ++j) e += sums[j];
    const double nn = norm[0];
    out[0] = e / nn;
    out[1] = nn;
  }
}

// out[i] = sum over the slots listed for output i, in list order
__global__ void __launch_bounds__(256) k_gather_slots(const double* __restrict__ slot_val,
                                                      const uint32_t* __restrict__ off,
                                                      const uint32_t* __restrict__ idx,
                                                      const double* __restrict__ weight, int n_out,
                                                      double* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_out) return;
  double s = 0.0;
  for (uint32_t k = off[i]; k < off[i + 1]; ++k) s += weight[k] * slot_val[idx[k]];
  out[i] = s;
}

__global__ void __launch_bounds__(256) k_fill_f64(double* __restrict__ p, uint64_t n, double v) {
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <typename T>
__global__ void __launch_bounds__(256) k_scale(T* __restrict__ psi, uint64_t n_amp, const double* __restrict__ norm2) {
  using R = typename Real<T>::type;
  const R f = R(1.0 / sqrt(norm2[0]));
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < n_amp; i += stride) {
    T v = psi[i];
    v.x *= f;
    if constexpr (!is_real_amp<T>) v.y *= f;
    psi[i] = v;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_gather_amps(const T* __restrict__ psi, const uint64_t* __restrict__ idx,
                                                     int64_t count, double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= count) return;
  const T v = psi[idx[i]];
  out[2 * i] = v.x;
  out[2 * i + 1] = v.y;
}

// ---------------------------------------------------------------------------
// Deflation (Eq. 12): H_eff = H + sum_j alpha_j |Psi_j><Psi_j|.  The adjoint
// needs lambda = H_eff psi = H psi + sum_j alpha_j <Psi_j|psi> Psi_j: one pass
// forms every overlap <Psi_j|psi> (psi read once, FP64 partials per block),
// a second adds the rank-one terms into lambda.
// ---------------------------------------------------------------------------
// partials[(2j) * grid + block] = Re <P_j|psi>, [(2j + 1) * grid + block] = Im
template <typename T>
__global__ void __launch_bounds__(256) k_overlaps(const T* __restrict__ psi, ProjArgs pa, uint64_t n_amp,
                                                  double* __restrict__ partials) {
  __shared__ double red[4];
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  double re[kMaxProj], im[kMaxProj];
#pragma unroll
  for (int j = 0; j < kMaxProj; ++j) re[j] = im[j] = 0.0;
  for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < n_amp; i += stride) {
    const T u = psi[i];
#pragma unroll
    for (int j = 0; j < kMaxProj; ++j) {
      if (j >= pa.k) break;
      const T v = static_cast<const T*>(pa.p[j])[i];
      re[j] += (double)v.x * u.x + (double)v.y * u.y;  // conj(v) u
      im[j] += (double)v.x * u.y - (double)v.y * u.x;
    }
  }
  for (int j = 0; j < pa.k; ++j) {
    const double a = block_sum<256>(re[j], red);
    if (threadIdx.x == 0) partials[uint64_t(2 * j) * gridDim.x + blockIdx.x] = a;
    const double b = block_sum<256>(im[j], red);
    if (threadIdx.x == 0) partials[uint64_t(2 * j + 1) * gridDim.x + blockIdx.x] = b;
  }
}

// lam += sum_j alpha_j ovl_j P_j, ovl = (re, im) pairs in device memory
template <typename T>
__global__ void __launch_bounds__(256) k_deflate(T* __restrict__ lam, ProjArgs pa, const double* __restrict__ ovl,
                                                 uint64_t n_amp) {
  using R = typename Real<T>::type;
  double cr[kMaxProj], ci[kMaxProj];
#pragma unroll
  for (int j = 0; j < kMaxProj; ++j) {
    cr[j] = j < pa.k ? pa.alpha[j] * ovl[2 * j] : 0.0;
    ci[j] = j < pa.k ? pa.alpha[j] * ovl[2 * j + 1] : 0.0;
  }
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < n_amp; i += stride) {
    T l = lam[i];
    double lr = l.x, li = l.y;
#pragma unroll
    for (int j = 0; j < kMaxProj; ++j) {
      if (j >= pa.k) break;
      const T v = static_cast<const T*>(pa.p[j])[i];
      lr += cr[j] * v.x - ci[j] * v.y;
      li += cr[j] * v.y + ci[j] * v.x;
    }
    l.x = R(lr);
    if constexpr (!is_real_amp<T>) l.y = R(li);
    lam[i] = l;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_dot(int dtype, const void* a, const void* b, const double* d, uint64_t n_amp, int grid,
                      double* partials, hipStream_t st) {
  return by_dtype(dtype, [&](auto tag) {
    using T = decltype(tag);
    hipLaunchKernelGGL((k_dot<T>), dim3(grid), dim3(256), 0, st, static_cast<const T*>(a), static_cast<const T*>(b), d,
                       n_amp, partials);
  });
}

hipError_t launch_imag_count(int dtype, const void* a, uint64_t n_amp, int grid, double* partials, hipStream_t st) {
  return by_dtype(dtype, [&](auto tag) {
    using T = decltype(tag);
    hipLaunchKernelGGL((k_imag_count<T>), dim3(grid), dim3(256), 0, st, static_cast<const T*>(a), n_amp, partials);
  });
}

hipError_t launch_amp_exponent(int dtype, const void* a, uint64_t n_amp, int grid, double* partials, hipStream_t st) {
  return by_dtype(dtype, [&](auto tag) {
    using T = decltype(tag);
    hipLaunchKernelGGL((k_amp_exponent<T>), dim3(grid), dim3(256), 0, st, static_cast<const T*>(a), n_amp, partials);
  });
}

hipError_t launch_reduce_rows(const double* in, uint64_t stride, uint32_t len, uint32_t rows, double* out,
                              hipStream_t st) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_rows, dim3(rows), dim3(256), 0, st, in, stride, len, out);
  return hipGetLastError();
}

hipError_t launch_finish_energy(const double* sums, int nh, const double* norm, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_finish_energy, dim3(1), dim3(64), 0, st, sums, nh, norm, out);
  return hipGetLastError();
}

hipError_t launch_gather_slots(const double* slot_val, const uint32_t* off, const uint32_t* idx,
                               const double* weight, int n_out, double* out, hipStream_t st) {
  if (n_out == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_slots, dim3((n_out + 255) / 256), dim3(256), 0, st, slot_val, off, idx, weight,
                     n_out, out);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, uint64_t n, double v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t want = (n + 255) / 256;
  const int grid = int(want < 4096 ? want : 4096);
  hipLaunchKernelGGL(k_fill_f64, dim3(grid), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_scale(int dtype, void* psi, uint64_t n_amp, const double* norm2, hipStream_t st) {
  const uint64_t want = (n_amp + 255) / 256;
  const int grid = int(want < 4096 ? want : 4096);
  return by_dtype(dtype, [&](auto tag) {
    using T = decltype(tag);
    hipLaunchKernelGGL((k_scale<T>), dim3(grid), dim3(256), 0, st, static_cast<T*>(psi), n_amp, norm2);
  });
}

hipError_t launch_gather_amps(int dtype, const void* psi, const uint64_t* idx, int64_t count, double* out,
                              hipStream_t st) {
  if (count == 0) return hipSuccess;
  const int grid = int((count + 255) / 256);
  return by_dtype(dtype, [&](auto tag) {
    using T = decltype(tag);
    hipLaunchKernelGGL((k_gather_amps<T>), dim3(grid), dim3(256), 0, st, static_cast<const T*>(psi), idx, count,
                       out);
  });
}

hipError_t launch_overlaps(int dtype, const void* psi, const ProjArgs& pa, uint64_t n_amp, int grid,
                           double* partials, hipStream_t st) {
  return by_dtype(dtype, [&](auto tag) {
    using T = decltype(tag);
    hipLaunchKernelGGL((k_overlaps<T>), dim3(grid), dim3(256), 0, st, static_cast<const T*>(psi), pa, n_amp,
                       partials);
  });
}

hipError_t launch_deflate(int dtype, void* lam, const ProjArgs& pa, const double* ovl, uint64_t n_amp, int grid,
                          hipStream_t st) {
  return by_dtype(dtype, [&](auto tag) {
    using T = decltype(tag);
    hipLaunchKernelGGL((k_deflate<T>), dim3(grid), dim3(256), 0, st, static_cast<T*>(lam), pa, ovl, n_amp);
  });
}

}  // namespace q2sv
