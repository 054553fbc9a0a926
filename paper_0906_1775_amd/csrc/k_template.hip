// Template columns B of the extended pointing [P B] ("Using MADmap" section
// of the MADmap paper, eqs. eDSN1 and PmatExt), and the white-noise weighting
// used when n_c = 1.
//
// One-hot templates (synchronous bins, destriping offsets) are pointing
// matrices of their own with one unit weight per row: the plan builds them
// with the pixel machinery (sort, observed compaction, sliced scatter) and
// only the gather into an existing TOD needs a kernel here.
//
// The half-wave-plate block (eq. HWPmat) has 32 dense columns per segment,
// evaluated on the fly from the polarizer angle w_t: for k = 1..8,
// cos(k w), tau cos(k w), sin(k w), tau sin(k w), with tau the sample index
// centred on the segment and scaled to (-1, 1).  cos(k w) and sin(k w) come
// from one sincos and the angle-addition recurrence, in float64.  Samples are
// cut into tiles of at most kTileSamples samples inside one segment; the scatter
// writes one partial sum per tile and column, and a second kernel adds the
// tiles of each segment in order (no atomics, fixed summation order).
#include "mm_internal.h"

namespace mm {

static dim3 grid_for(int64_t n) {
  int64_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  if (nb < 1) nb = 1;
  return dim3((unsigned)nb);
}

// ---------------------------------------------------------------- one-hot gather
template <typename Ty>
__global__ void k_onehot_gather(const int32_t* __restrict__ obs_idx, const double* __restrict__ p,
                                int64_t vs, int64_t off, Ty* __restrict__ y, int64_t n_t, int n_rhs,
                                const CgState* __restrict__ st) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_t; t += stride) {
    const int32_t o = obs_idx[t];
    if (o < 0) continue;
    for (int r = 0; r < n_rhs; ++r) {
      if (st && !st[r].active) continue;
      const int64_t i = (int64_t)r * n_t + t;
      y[i] = (Ty)((double)y[i] + p[(int64_t)r * vs + off + o]);
    }
  }
}

hipError_t launch_onehot_gather(bool y_f64, const int32_t* obs_idx, const double* p, int64_t vs, int64_t off,
                                void* y, int64_t n_t, int n_rhs, hipStream_t s, const CgState* st) {
  if (n_t == 0) return hipSuccess;
  if (y_f64) hipLaunchKernelGGL(k_onehot_gather<double>, grid_for(n_t), dim3(256), 0, s, obs_idx, p, vs, off, (double*)y, n_t, n_rhs, st);
  else hipLaunchKernelGGL(k_onehot_gather<float>, grid_for(n_t), dim3(256), 0, s, obs_idx, p, vs, off, (float*)y, n_t, n_rhs, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------- HWP block
__device__ __forceinline__ void hwp_harmonics(float w, double* c, double* sn) {
  double s1, c1;
  sincos((double)w, &s1, &c1);
  c[0] = c1;
  sn[0] = s1;
#pragma unroll
  for (int k = 1; k < kHwpHarmonics; ++k) {
    c[k] = c[k - 1] * c1 - sn[k - 1] * s1;
    sn[k] = sn[k - 1] * c1 + c[k - 1] * s1;
  }
}

__device__ __forceinline__ double hwp_tau(int64_t t, int64_t s0, double L) {
  return (2.0 * (double)(t - s0) - (L - 1.0)) / L;
}

// y[r][t] += sum_i C[t][i] a[r][seg(t)][i] over the tiles
template <typename Ty>
__global__ __launch_bounds__(256) void k_hwp_gather(const SampleTile* __restrict__ tiles,
                                                    const int64_t* __restrict__ seg_start,
                                                    const float* __restrict__ omega, const double* __restrict__ p,
                                                    int64_t vs, int64_t off, Ty* __restrict__ y, int64_t n_t,
                                                    int n_rhs, const CgState* __restrict__ st) {
  __shared__ double a[kMaxRhs][kHwpColumns];
  const SampleTile T = tiles[blockIdx.x];
  for (int i = threadIdx.x; i < n_rhs * kHwpColumns; i += blockDim.x)
    a[i / kHwpColumns][i % kHwpColumns] = p[(int64_t)(i / kHwpColumns) * vs + off +
                                            (int64_t)T.id * kHwpColumns + i % kHwpColumns];
  __syncthreads();
  const int64_t s0 = seg_start[T.id];
  const double L = (double)(seg_start[T.id + 1] - s0);
  for (int64_t t = T.t0 + threadIdx.x; t < T.t1; t += blockDim.x) {
    double c[kHwpHarmonics], sn[kHwpHarmonics];
    hwp_harmonics(omega[t], c, sn);
    const double tau = hwp_tau(t, s0, L);
    for (int r = 0; r < n_rhs; ++r) {
      if (st && !st[r].active) continue;
      const double* ar = a[r];
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < kHwpHarmonics; ++k)
        v += (ar[k] + tau * ar[8 + k]) * c[k] + (ar[16 + k] + tau * ar[24 + k]) * sn[k];
      const int64_t i = (int64_t)r * n_t + t;
      y[i] = (Ty)((double)y[i] + v);
    }
  }
}

hipError_t launch_hwp_gather(bool y_f64, const SampleTile* tiles, int n_tiles, const int64_t* seg_start,
                             const float* omega, const double* p, int64_t vs, int64_t off, void* y, int64_t n_t,
                             int n_rhs, hipStream_t s, const CgState* st) {
  if (n_tiles == 0) return hipSuccess;
  if (n_rhs > kMaxRhs) return hipErrorInvalidValue;
  if (y_f64) hipLaunchKernelGGL(k_hwp_gather<double>, dim3(n_tiles), dim3(256), 0, s, tiles, seg_start, omega, p, vs, off, (double*)y, n_t, n_rhs, st);
  else hipLaunchKernelGGL(k_hwp_gather<float>, dim3(n_tiles), dim3(256), 0, s, tiles, seg_start, omega, p, vs, off, (float*)y, n_t, n_rhs, st);
  return hipGetLastError();
}

// white-noise weight f_b(0) of sample t (interval by binary search; plan time only)
__device__ __forceinline__ double white_weight(int64_t t, const int64_t* __restrict__ iv_start, int n_iv,
                                               const int32_t* __restrict__ iv_filter,
                                               const double* __restrict__ lags, int n_c) {
  int lo = 0, hi = n_iv;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (iv_start[mid] <= t) lo = mid; else hi = mid;
  }
  return lags[(int64_t)iv_filter[lo] * n_c];
}

// partial[tile][r][i] = sum over the tile of C[t][i] y[r][t]            (mode 0)
// partial[tile][0][i] = sum over the tile of C[t][i]^2 w(t)             (mode 1: w = f_b(0);
//                                                                        mode 2: w = 1)
template <typename Ty>
__global__ __launch_bounds__(256) void k_hwp_scatter(const SampleTile* __restrict__ tiles,
                                                     const int64_t* __restrict__ seg_start,
                                                     const float* __restrict__ omega, const Ty* __restrict__ y,
                                                     int64_t n_t, int n_rhs, double* __restrict__ partial, int mode,
                                                     const int64_t* __restrict__ iv_start, int n_iv,
                                                     const int32_t* __restrict__ iv_filter,
                                                     const double* __restrict__ lags, int n_c,
                                                     const CgState* __restrict__ st) {
  __shared__ double red[256 / 64][kHwpColumns];
  const SampleTile T = tiles[blockIdx.x];
  const int64_t s0 = seg_start[T.id];
  const double L = (double)(seg_start[T.id + 1] - s0);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int R = mode == 0 ? n_rhs : 1;
  for (int r = 0; r < R; ++r) {
    if (st && !st[r].active) continue;     // uniform over the block
    double acc[kHwpColumns];
#pragma unroll
    for (int i = 0; i < kHwpColumns; ++i) acc[i] = 0.0;
    for (int64_t t = T.t0 + threadIdx.x; t < T.t1; t += blockDim.x) {
      double c[kHwpHarmonics], sn[kHwpHarmonics];
      hwp_harmonics(omega[t], c, sn);
      const double tau = hwp_tau(t, s0, L);
      if (mode == 0) {
        const double v = (double)y[(int64_t)r * n_t + t];
        const double tv = tau * v;
#pragma unroll
        for (int k = 0; k < kHwpHarmonics; ++k) {
          acc[k] += c[k] * v;
          acc[8 + k] += c[k] * tv;
          acc[16 + k] += sn[k] * v;
          acc[24 + k] += sn[k] * tv;
        }
      } else {
        const double w = mode == 1 ? white_weight(t, iv_start, n_iv, iv_filter, lags, n_c) : 1.0;
        const double t2w = tau * tau * w;
#pragma unroll
        for (int k = 0; k < kHwpHarmonics; ++k) {
          acc[k] += c[k] * c[k] * w;
          acc[8 + k] += c[k] * c[k] * t2w;
          acc[16 + k] += sn[k] * sn[k] * w;
          acc[24 + k] += sn[k] * sn[k] * t2w;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kHwpColumns; ++i) {
      double v = acc[i];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) red[wv][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < kHwpColumns) {
      double v = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += red[w][threadIdx.x];
      partial[((int64_t)blockIdx.x * R + r) * kHwpColumns + threadIdx.x] = v;
    }
    __syncthreads();
  }
}

// q[r][off + 32 g + i] = sum over the tiles of segment g (in order) of partial[tile][r][i];
// with p, also pq_part[r * pq_stride + pq_slot] = sum of p q over the block (fixed order)
__global__ __launch_bounds__(256) void k_hwp_reduce(const double* __restrict__ partial,
                                                    const int32_t* __restrict__ seg_tile, int n_seg, int n_rhs,
                                                    double* __restrict__ q, int64_t vs, int64_t off,
                                                    const double* __restrict__ p, double* __restrict__ pq_part,
                                                    int pq_stride, int pq_slot, const CgState* __restrict__ st) {
  __shared__ double sh[256 / 64];
  const int r = blockIdx.x;
  if (st && !st[r].active) return;
  double pq = 0.0;
  for (int64_t j = threadIdx.x; j < (int64_t)n_seg * kHwpColumns; j += blockDim.x) {
    const int g = (int)(j / kHwpColumns), i = (int)(j % kHwpColumns);
    double v = 0.0;
    for (int tl = seg_tile[g]; tl < seg_tile[g + 1]; ++tl)
      v += partial[((int64_t)tl * n_rhs + r) * kHwpColumns + i];
    const int64_t e = (int64_t)r * vs + off + j;
    q[e] = v;
    if (p) pq += p[e] * v;
  }
  if (p) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) pq += __shfl_xor(pq, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = pq;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
      pq_part[(int64_t)r * pq_stride + pq_slot] = s;
    }
  }
}

hipError_t launch_hwp_scatter(bool y_f64, const SampleTile* tiles, int n_tiles, const int32_t* seg_tile, int n_seg,
                              const int64_t* seg_start, const float* omega, const void* y, int64_t n_t, int n_rhs,
                              double* partial, double* q, int64_t vs, int64_t off, const double* p,
                              double* pq_part, int pq_stride, int pq_slot, hipStream_t s, const CgState* st) {
  if (n_seg == 0) return hipSuccess;
  if (n_tiles > 0) {
    if (y_f64)
      hipLaunchKernelGGL(k_hwp_scatter<double>, dim3(n_tiles), dim3(256), 0, s, tiles, seg_start, omega,
                         (const double*)y, n_t, n_rhs, partial, 0, nullptr, 0, nullptr, nullptr, 1, st);
    else
      hipLaunchKernelGGL(k_hwp_scatter<float>, dim3(n_tiles), dim3(256), 0, s, tiles, seg_start, omega,
                         (const float*)y, n_t, n_rhs, partial, 0, nullptr, 0, nullptr, nullptr, 1, st);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_hwp_reduce, dim3(n_rhs), dim3(256), 0, s, partial, seg_tile, n_seg, n_rhs, q, vs, off, p,
                     pq_part, pq_stride, pq_slot, st);
  return hipGetLastError();
}

// diag[32 g + i] = sum over segment g of C[t][i]^2 w(t) (w = f_b(0) for kind 0, 1 for kind 1)
hipError_t launch_hwp_diag(int kind, const SampleTile* tiles, int n_tiles, const int32_t* seg_tile, int n_seg,
                           const int64_t* seg_start, const float* omega, const int64_t* iv_start, int n_iv,
                           const int32_t* iv_filter, const double* lags, int n_c, double* partial,
                           double* diag, hipStream_t s) {
  if (n_seg == 0) return hipSuccess;
  if (n_tiles > 0) {
    hipLaunchKernelGGL(k_hwp_scatter<float>, dim3(n_tiles), dim3(256), 0, s, tiles, seg_start, omega,
                       (const float*)nullptr, (int64_t)0, 1, partial, kind == 0 ? 1 : 2, iv_start, n_iv, iv_filter,
                       lags, n_c, (const CgState*)nullptr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_hwp_reduce, dim3(1), dim3(256), 0, s, partial, seg_tile, n_seg, 1, diag, (int64_t)0,
                     (int64_t)0, (const double*)nullptr, (double*)nullptr, 0, 0, (const CgState*)nullptr);
  return hipGetLastError();
}

// ---------------------------------------------------------------- diagonal helpers
// out[j] = 1 / d[j] where d[j] > 0, else 0
__global__ void k_invert_diag(const double* __restrict__ d, double* __restrict__ out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride)
    out[j] = d[j] > 0.0 ? 1.0 / d[j] : 0.0;
}

hipError_t launch_invert_diag(const double* d, double* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_invert_diag, grid_for(n), dim3(256), 0, s, d, out, n);
  return hipGetLastError();
}

// dst[r][i] = src[r][i], i < n, rows of stride dst_stride / src_stride
__global__ void k_copy_rows(const double* __restrict__ src, int64_t src_stride, double* __restrict__ dst,
                            int64_t dst_stride, int64_t n, int n_rhs) {
  const int64_t total = n * n_rhs;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += stride) {
    const int64_t r = k / n, i = k % n;
    dst[r * dst_stride + i] = src[r * src_stride + i];
  }
}

hipError_t launch_copy_rows(const double* src, int64_t src_stride, double* dst, int64_t dst_stride, int64_t n,
                            int n_rhs, hipStream_t s) {
  if (n == 0 || n_rhs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_rows, grid_for(n * n_rhs), dim3(256), 0, s, src, src_stride, dst, dst_stride, n, n_rhs);
  return hipGetLastError();
}

// ---------------------------------------------------------------- white noise
// y_out[r][t] = f_b(0) y_in[r][t] over tiles that each lie inside one interval
template <typename Ti, typename To>
__global__ __launch_bounds__(256) void k_white(const SampleTile* __restrict__ tiles, const int32_t* __restrict__ iv_filter,
                                               const double* __restrict__ lags, int n_c, const Ti* __restrict__ y_in,
                                               To* __restrict__ y_out, int64_t n_t, const CgState* __restrict__ st) {
  const SampleTile T = tiles[blockIdx.x];
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  const double f0 = lags[(int64_t)iv_filter[T.id] * n_c];
  const Ti* yi = y_in + (int64_t)r * n_t;
  To* yo = y_out + (int64_t)r * n_t;
  for (int64_t t = T.t0 + threadIdx.x; t < T.t1; t += blockDim.x) yo[t] = (To)(f0 * (double)yi[t]);
}

hipError_t launch_white(bool out_f64, bool in_f64, const SampleTile* tiles, int n_tiles, const int32_t* iv_filter,
                        const double* lags, int n_c, const void* y_in, void* y_out, int64_t n_t, int n_rhs,
                        hipStream_t s, const CgState* st) {
  if (n_tiles == 0) return hipSuccess;
  const dim3 g(n_tiles, n_rhs), b(256);
  if (in_f64 && out_f64) hipLaunchKernelGGL((k_white<double, double>), g, b, 0, s, tiles, iv_filter, lags, n_c, (const double*)y_in, (double*)y_out, n_t, st);
  else if (in_f64) hipLaunchKernelGGL((k_white<double, float>), g, b, 0, s, tiles, iv_filter, lags, n_c, (const double*)y_in, (float*)y_out, n_t, st);
  else if (out_f64) hipLaunchKernelGGL((k_white<float, double>), g, b, 0, s, tiles, iv_filter, lags, n_c, (const float*)y_in, (double*)y_out, n_t, st);
  else hipLaunchKernelGGL((k_white<float, float>), g, b, 0, s, tiles, iv_filter, lags, n_c, (const float*)y_in, (float*)y_out, n_t, st);
  return hipGetLastError();
}

}  // namespace mm
