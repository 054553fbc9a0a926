// Pointing operators P (gather, map -> TOD) and P^T (scatter-add, TOD -> map).
//
// Formalism section of the MADmap paper: the row of sample t of P holds one
// unit weight for temperature, or (1/2, sin(2a_t)/2, cos(2a_t)/2) in the
// (I, Q, U) columns of its pixel for an ideal polarimeter; rows of excised
// samples are zero.
//
// Gather streams the time-ordered pointing (observed pixel id, sin/cos pair)
// coalesced and reads the map through the caches.  Scatter walks the
// pixel-major copy of the pointing built by the plan: a group of G lanes owns
// one pixel, strides over that pixel's samples and reduces across the group
// with cross-lane shuffles, so every pixel sum is formed in a fixed order by
// one group and no atomics are needed.  Maps are float64 [R][n_obs][ns].
#include "mm_internal.h"

namespace mm {

template <typename Ty, int NS>
__global__ void k_gather(const int32_t* __restrict__ pix_obs, const float2* __restrict__ w,
                         const double* __restrict__ p, Ty* __restrict__ y, int64_t n_t,
                         int64_t n_obs, int n_rhs) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_t; t += stride) {
    const int32_t o = pix_obs[t];
    if (NS == 1) {
      for (int r = 0; r < n_rhs; ++r)
        y[(int64_t)r * n_t + t] = o >= 0 ? (Ty)p[(int64_t)r * n_obs + o] : (Ty)0;
    } else {
      const float2 sc = w[t];
      const double s = sc.x, c = sc.y;
      for (int r = 0; r < n_rhs; ++r) {
        double v = 0.0;
        if (o >= 0) {
          const double* m = p + ((int64_t)r * n_obs + o) * 3;
          v = 0.5 * (m[0] + s * m[1] + c * m[2]);
        }
        y[(int64_t)r * n_t + t] = (Ty)v;
      }
    }
  }
}

hipError_t launch_gather(bool out_f64, int ns, const int32_t* pix_obs, const float* w,
                         const double* p, void* y, int64_t n_t, int64_t n_obs, int n_rhs,
                         hipStream_t s) {
  if (n_t == 0) return hipSuccess;
  int64_t nb = (n_t + 255) / 256;
  if (nb > 65536) nb = 65536;
  const dim3 g((unsigned)nb), b(256);
  const float2* w2 = (const float2*)w;
  if (out_f64) {
    if (ns == 1) hipLaunchKernelGGL((k_gather<double, 1>), g, b, 0, s, pix_obs, w2, p, (double*)y, n_t, n_obs, n_rhs);
    else hipLaunchKernelGGL((k_gather<double, 3>), g, b, 0, s, pix_obs, w2, p, (double*)y, n_t, n_obs, n_rhs);
  } else {
    if (ns == 1) hipLaunchKernelGGL((k_gather<float, 1>), g, b, 0, s, pix_obs, w2, p, (float*)y, n_t, n_obs, n_rhs);
    else hipLaunchKernelGGL((k_gather<float, 3>), g, b, 0, s, pix_obs, w2, p, (float*)y, n_t, n_obs, n_rhs);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- scatter
// Accumulator: plain float64 sums for float64 TOD; for float32 TOD the
// products are formed in float32 and summed with Neumaier's compensated
// summation in float32, and the (sum, compensation) pair is folded to float64
// before the cross-lane reduction.
template <typename Ty> struct Acc;
template <> struct Acc<double> {
  double s = 0.0;
  __device__ void add(double x) { s += x; }
  __device__ double value() const { return s; }
};
template <> struct Acc<float> {
  float s = 0.0f, c = 0.0f;
  __device__ void add(float x) {
    const float t = s + x;
    if (fabsf(s) >= fabsf(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
  }
  __device__ double value() const { return (double)s + (double)c; }
};

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

template <typename Ty, int NS, int G>
__global__ void k_scatter(const int64_t* __restrict__ pix_ptr, const int32_t* __restrict__ perm,
                          const float2* __restrict__ w_pm, const Ty* __restrict__ y,
                          double* __restrict__ q, int64_t n_obs, int64_t n_t, int n_rhs) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t o = gid / G;
  const int lane = (int)(gid % G);
  const bool ok = o < n_obs;   // whole groups share o, so shuffles stay within live lanes
  const int64_t k0 = ok ? pix_ptr[o] : 0, k1 = ok ? pix_ptr[o + 1] : 0;
  for (int r = 0; r < n_rhs; ++r) {
    const Ty* __restrict__ yr = y + (int64_t)r * n_t;
    Acc<Ty> a0, a1, a2;
    for (int64_t k = k0 + lane; k < k1; k += G) {
      const Ty v = yr[perm[k]];
      if (NS == 1) {
        a0.add(v);
      } else {
        const float2 sc = w_pm[k];
        const Ty h = (Ty)0.5 * v;
        a0.add(h);
        a1.add(h * (Ty)sc.x);
        a2.add(h * (Ty)sc.y);
      }
    }
    const double s0 = group_sum<G>(a0.value());
    if (NS == 1) {
      if (ok && lane == 0) q[(int64_t)r * n_obs + o] = s0;
    } else {
      const double s1 = group_sum<G>(a1.value());
      const double s2 = group_sum<G>(a2.value());
      if (ok && lane == 0) {
        double* d = q + ((int64_t)r * n_obs + o) * 3;
        d[0] = s0;
        d[1] = s1;
        d[2] = s2;
      }
    }
  }
}

template <typename Ty, int NS>
static hipError_t scatter_g(int group, dim3 g, hipStream_t s, const int64_t* pp, const int32_t* perm,
                            const float2* w, const Ty* y, double* q, int64_t n_obs, int64_t n_t,
                            int n_rhs) {
  const dim3 b(256);
  switch (group) {
    case 4: hipLaunchKernelGGL((k_scatter<Ty, NS, 4>), g, b, 0, s, pp, perm, w, y, q, n_obs, n_t, n_rhs); break;
    case 8: hipLaunchKernelGGL((k_scatter<Ty, NS, 8>), g, b, 0, s, pp, perm, w, y, q, n_obs, n_t, n_rhs); break;
    case 16: hipLaunchKernelGGL((k_scatter<Ty, NS, 16>), g, b, 0, s, pp, perm, w, y, q, n_obs, n_t, n_rhs); break;
    case 32: hipLaunchKernelGGL((k_scatter<Ty, NS, 32>), g, b, 0, s, pp, perm, w, y, q, n_obs, n_t, n_rhs); break;
    case 64: hipLaunchKernelGGL((k_scatter<Ty, NS, 64>), g, b, 0, s, pp, perm, w, y, q, n_obs, n_t, n_rhs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_scatter(bool in_f64, int ns, int group, const int64_t* pix_ptr,
                          const int32_t* perm, const float* w_pm, const void* y, double* q,
                          int64_t n_obs, int64_t n_t, int n_rhs, hipStream_t s) {
  if (n_obs == 0) return hipSuccess;
  const int64_t threads = n_obs * group;
  const dim3 g((unsigned)((threads + 255) / 256));
  const float2* w = (const float2*)w_pm;
  if (in_f64)
    return ns == 1 ? scatter_g<double, 1>(group, g, s, pix_ptr, perm, w, (const double*)y, q, n_obs, n_t, n_rhs)
                   : scatter_g<double, 3>(group, g, s, pix_ptr, perm, w, (const double*)y, q, n_obs, n_t, n_rhs);
  return ns == 1 ? scatter_g<float, 1>(group, g, s, pix_ptr, perm, w, (const float*)y, q, n_obs, n_t, n_rhs)
                 : scatter_g<float, 3>(group, g, s, pix_ptr, perm, w, (const float*)y, q, n_obs, n_t, n_rhs);
}

// ---------------------------------------------------------------- layout helpers
template <typename Ti, typename To>
__global__ void k_convert(const Ti* __restrict__ in, To* __restrict__ out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = (To)in[i];
}

static dim3 grid_for(int64_t n) {
  int64_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  if (nb < 1) nb = 1;
  return dim3((unsigned)nb);
}

hipError_t launch_convert(bool in_f64, bool out_f64, const void* in, void* out, int64_t n,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 g = grid_for(n), b(256);
  if (in_f64 && out_f64) hipLaunchKernelGGL((k_convert<double, double>), g, b, 0, s, (const double*)in, (double*)out, n);
  else if (in_f64) hipLaunchKernelGGL((k_convert<double, float>), g, b, 0, s, (const double*)in, (float*)out, n);
  else if (out_f64) hipLaunchKernelGGL((k_convert<float, double>), g, b, 0, s, (const float*)in, (double*)out, n);
  else hipLaunchKernelGGL((k_convert<float, float>), g, b, 0, s, (const float*)in, (float*)out, n);
  return hipGetLastError();
}

__global__ void k_to_observed(const double* __restrict__ glob, double* __restrict__ obs,
                              const int32_t* __restrict__ obs2glob, int64_t n_obs, int64_t n_pix,
                              int ns, int n_rhs) {
  const int64_t n = n_obs * ns * n_rhs;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int64_t per = n_obs * ns;
    const int64_t r = i / per, rem = i % per, o = rem / ns, c = rem % ns;
    obs[i] = glob[(r * n_pix + obs2glob[o]) * ns + c];
  }
}

// global map = observed values at observed pixels, 0 elsewhere (one pass over the global map)
__global__ void k_to_global(const double* __restrict__ obs, double* __restrict__ glob,
                            const int32_t* __restrict__ obs2glob, int64_t n_obs, int64_t n_pix,
                            int ns, int n_rhs) {
  const int64_t n = n_pix * n_rhs;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int64_t r = i / n_pix, gp = i % n_pix;
    // binary search of gp in the sorted obs2glob
    int64_t lo = 0, hi = n_obs;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (obs2glob[mid] < gp) lo = mid + 1; else hi = mid;
    }
    const bool seen = lo < n_obs && obs2glob[lo] == gp;
    for (int c = 0; c < ns; ++c)
      glob[i * ns + c] = seen ? obs[(r * n_obs + lo) * ns + c] : 0.0;
  }
}

hipError_t launch_to_observed(const double* glob, double* obs, const int32_t* obs2glob,
                              int64_t n_obs, int64_t n_pix, int ns, int n_rhs, hipStream_t s) {
  const int64_t n = n_obs * ns * n_rhs;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_observed, grid_for(n), dim3(256), 0, s, glob, obs, obs2glob, n_obs, n_pix, ns, n_rhs);
  return hipGetLastError();
}

hipError_t launch_to_global(const double* obs, double* glob, const int32_t* obs2glob,
                            int64_t n_obs, int64_t n_pix, int ns, int n_rhs, hipStream_t s) {
  const int64_t n = n_pix * n_rhs;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_global, grid_for(n), dim3(256), 0, s, obs, glob, obs2glob, n_obs, n_pix, ns, n_rhs);
  return hipGetLastError();
}

__global__ void k_hits(const int64_t* __restrict__ pix_ptr, const int32_t* __restrict__ obs2glob,
                       int32_t* __restrict__ hits, int64_t n_obs, int64_t n_pix) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pix; i += stride) {
    int64_t lo = 0, hi = n_obs;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (obs2glob[mid] < i) lo = mid + 1; else hi = mid;
    }
    hits[i] = (lo < n_obs && obs2glob[lo] == i) ? (int32_t)(pix_ptr[lo + 1] - pix_ptr[lo]) : 0;
  }
}

hipError_t launch_hits(const int64_t* pix_ptr, const int32_t* obs2glob, int32_t* hits,
                       int64_t n_obs, int64_t n_pix, hipStream_t s) {
  if (n_pix == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hits, grid_for(n_pix), dim3(256), 0, s, pix_ptr, obs2glob, hits, n_obs, n_pix);
  return hipGetLastError();
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, T v, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<double>, grid_for(n), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<int32_t>, grid_for(n), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace mm
