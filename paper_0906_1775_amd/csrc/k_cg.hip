// Preconditioned conjugate-gradient vector kernels and the block
// preconditioner (Implementation section of the MADmap paper).
//
// All pixel-domain vectors are float64 rows [R][vs]: n_obs blocks of ns
// pixel values, then the template amplitudes (diagonal preconditioner).  Dot products are
// formed as kDotBlocks partial sums per RHS (fixed grid => fixed summation
// order => bitwise repeatable) and folded by the scalar kernels, which keep
// every CG scalar on the device (CgState), so an iteration needs no host
// round trip.
//
// Iteration (per RHS, while active), matching the textbook PCG order:
//   q = H p;  alpha = rho / (p.q);  x += alpha p;  r -= alpha q;
//   rel = ||r|| / ||b||;  keep x if rel is the lowest so far;  stop if rel <= tol;
//   z = M r;  rho' = r.z;  beta = rho'/rho;  p = z + beta p.
#include "mm_internal.h"

namespace mm {

static dim3 grid_for(int64_t n) {
  int64_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  if (nb < 1) nb = 1;
  return dim3((unsigned)nb);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  }
  __syncthreads();
  return s;   // valid in thread 0
}

// sum of the kDotBlocks partials of RHS r by one wavefront (fixed order)
__device__ __forceinline__ double fold_partials(const double* __restrict__ part, int r) {
  const int lane = threadIdx.x & 63;
  double v = 0.0;
  for (int i = lane; i < kDotBlocks; i += 64) v += part[(int64_t)r * kDotBlocks + i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------- dots
__global__ __launch_bounds__(kDotThreads) void k_dot(const double* __restrict__ x,
                                                     const double* __restrict__ y, int64_t nu,
                                                     double* __restrict__ partial) {
  __shared__ double sh[kDotThreads / 64];
  const int r = blockIdx.y;
  const double* xr = x + (int64_t)r * nu;
  const double* yr = y + (int64_t)r * nu;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < nu;
       i += (int64_t)kDotBlocks * kDotThreads)
    acc += xr[i] * yr[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[(int64_t)r * kDotBlocks + blockIdx.x] = s;
}

hipError_t launch_dot(const double* x, const double* y, int64_t nu, int n_rhs, double* partial,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_dot, dim3(kDotBlocks, n_rhs), dim3(kDotThreads), 0, s, x, y, nu, partial);
  return hipGetLastError();
}

// ---------------------------------------------------------------- scalars
__global__ void k_cg_init(CgState* st, const double* __restrict__ pbb, const double* __restrict__ prr,
                          const double* __restrict__ prz, double tol, int fixed,
                          double* __restrict__ history, int hist_stride) {
  const int r = blockIdx.x;
  const double bb = fold_partials(pbb, r);
  const double rr = fold_partials(prr, r);
  const double rz = fold_partials(prz, r);
  if (threadIdx.x != 0) return;
  CgState s;
  s.bnorm = sqrt(bb);
  s.rel = s.bnorm > 0.0 ? sqrt(rr) / s.bnorm : 0.0;
  s.rho = rz;
  s.alpha = 0.0;
  s.beta = 0.0;
  s.best_rel = s.rel;
  s.tol = tol;
  s.iter = 0;
  s.best_iter = 0;
  s.fixed = fixed;
  s.active = (s.bnorm > 0.0) && (fixed || !(s.rel <= tol)) ? 1 : 0;
  s.copy_best = 0;
  s.breakdown = 0;
  s.xcur = 0;
  s.xbest = 0;
  st[r] = s;
  if (history) history[(int64_t)r * hist_stride] = s.rel;
}

hipError_t launch_cg_init(CgState* st, const double* partial_bb, const double* partial_rr,
                          const double* partial_rz, double tol, int fixed, int n_rhs,
                          double* history, int hist_stride, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_init, dim3(n_rhs), dim3(64), 0, s, st, partial_bb, partial_rr, partial_rz,
                     tol, fixed, history, hist_stride);
  return hipGetLastError();
}

template <int NS>
__device__ __forceinline__ void precond_apply(const double* __restrict__ m, const double* r, double* z) {
  if (NS == 1) {
    z[0] = m[0] * r[0];
  } else {
    z[0] = m[0] * r[0] + m[1] * r[1] + m[2] * r[2];
    z[1] = m[1] * r[0] + m[3] * r[1] + m[4] * r[2];
    z[2] = m[2] * r[0] + m[4] * r[1] + m[5] * r[2];
  }
}

// Each block folds the p.q partial sums of the scatter in the same fixed
// order, so every block derives the same alpha; block 0 records it.
// One block walks a fixed set of pixels for a group of RG right-hand sides, so a
// pixel's preconditioner block is read once per group instead of once per RHS;
// every RHS's partial sums keep the order of a one-RHS pass (tail entries, then
// pixels, in grid-stride order).  Tv: the element type of q and z (float32 in the
// mixed-precision iteration: q as the scatter rounded it, z rounded after r.z is
// formed from its float64 value).  x += alpha p is left to the step kernel, which reads
// p anyway.
template <int NS, int RG, typename Tv>
__global__ __launch_bounds__(kDotThreads) void k_cg_update(
    double* __restrict__ rv, const Tv* __restrict__ q, Tv* __restrict__ z, const double* __restrict__ minv,
    CgState* __restrict__ st, CgState* __restrict__ st_prev, int64_t n_obs, int64_t vs,
    const double* __restrict__ minv_t, int64_t n_tail, int n_rhs, const double* __restrict__ pq_part, int n_pq,
    double* __restrict__ prz, double* __restrict__ prr) {
  __shared__ double sh[kDotThreads / 64];
  __shared__ double s_alpha[RG];
  constexpr int NM = NS == 1 ? 1 : 6;
  const int r0 = blockIdx.y * RG;
  const int tid = threadIdx.x;
  bool act[RG];
  double alpha[RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const int r = r0 + g;
    if (r >= n_rhs) {               // uniform over the block
      act[g] = false;
      alpha[g] = 0.0;
      continue;
    }
    double acc = 0.0;
    for (int i = tid; i < n_pq; i += kDotThreads) acc += pq_part[(int64_t)r * n_pq + i];
    const double pq = block_sum(acc, sh);
    const bool was_active = st[r].active != 0;
    if (tid == 0) {
      double al = 0.0;
      bool brk = false;
      if (was_active) {
        if (pq > 0.0 && isfinite(pq)) al = st[r].rho / pq;
        else brk = true;
      }
      s_alpha[g] = al;
      if (blockIdx.x == 0) {
        CgState v = st[r];
        v.alpha = al;
        v.breakdown = brk ? 1 : 0;
        st[r].alpha = al;            // read by no other block of this kernel
        st[r].breakdown = v.breakdown;
        st_prev[r] = v;              // the state before the step, for the scalar step that follows
      }
    }
    __syncthreads();
    alpha[g] = s_alpha[g];
    act[g] = was_active && alpha[g] != 0.0;
  }
  double arz[RG], arr[RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) arz[g] = arr[g] = 0.0;
  // template amplitudes (diagonal preconditioner)
  for (int64_t j = (int64_t)blockIdx.x * kDotThreads + tid; j < n_tail; j += (int64_t)kDotBlocks * kDotThreads) {
    const double mt = minv_t[j];
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      if (!act[g]) continue;
      const int64_t b = (int64_t)(r0 + g) * vs + n_obs * NS + j;
      const double rr = rv[b] - alpha[g] * (double)q[b];
      rv[b] = rr;
      const double zz = mt * rr;
      z[b] = (Tv)zz;
      arz[g] += rr * zz;
      arr[g] += rr * rr;
    }
  }
  for (int64_t o = (int64_t)blockIdx.x * kDotThreads + tid; o < n_obs; o += (int64_t)kDotBlocks * kDotThreads) {
    double m[NM];
#pragma unroll
    for (int k = 0; k < NM; ++k) m[k] = minv[o * NM + k];
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      if (!act[g]) continue;
      const int64_t b = (int64_t)(r0 + g) * vs + o * NS;
      double rr[NS], zz[NS];
#pragma unroll
      for (int c = 0; c < NS; ++c) {
        rr[c] = rv[b + c] - alpha[g] * (double)q[b + c];
        rv[b + c] = rr[c];
      }
      precond_apply<NS>(m, rr, zz);
#pragma unroll
      for (int c = 0; c < NS; ++c) {
        z[b + c] = (Tv)zz[c];
        arz[g] += rr[c] * zz[c];
        arr[g] += rr[c] * rr[c];
      }
    }
  }
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    if (r0 + g >= n_rhs) break;     // uniform over the block
    const double s1 = block_sum(arz[g], sh);
    const double s2 = block_sum(arr[g], sh);
    if (tid == 0) {
      prz[(int64_t)(r0 + g) * kDotBlocks + blockIdx.x] = s1;
      prr[(int64_t)(r0 + g) * kDotBlocks + blockIdx.x] = s2;
    }
  }
}

hipError_t launch_cg_update(int ns, double* r, const void* q, void* z,
                            bool qz_f32, const double* minv, CgState* st, CgState* st_prev, int64_t n_obs,
                            int64_t vs, const double* minv_t, int64_t n_tail,
                            int n_rhs, const double* pq_part, int n_pq, double* partial_rz,
                            double* partial_rr, hipStream_t s) {
  const dim3 b(kDotThreads);
#define MM_UPD(NS, RG, TV)                                                                                \
  hipLaunchKernelGGL((k_cg_update<NS, RG, TV>), dim3(kDotBlocks, (n_rhs + RG - 1) / RG), b, 0, s, r, \
                     (const TV*)q, (TV*)z, minv, st, st_prev, n_obs, vs, minv_t, n_tail, n_rhs, pq_part, n_pq,   \
                     partial_rz, partial_rr)
#define MM_UPD_T(TV)                                     \
  if (n_rhs == 1) {                                      \
    if (ns == 1) MM_UPD(1, 1, TV); else MM_UPD(3, 1, TV); \
  } else {                                               \
    if (ns == 1) MM_UPD(1, 8, TV); else MM_UPD(3, 8, TV); \
  }
  if (qz_f32) { MM_UPD_T(float) } else { MM_UPD_T(double) }
#undef MM_UPD_T
#undef MM_UPD
  return hipGetLastError();
}

// The scalar step of RHS s after an update: iteration count, relative residual,
// best iterate, convergence, beta and rho from the folded r.z and r.r.  Returns
// false when no step was taken (stopped, or p.q <= 0).
__device__ __forceinline__ bool cg_scalar_step(CgState& s, double rz, double rr) {
  if (!s.active || s.breakdown) {
    s.copy_best = 0;
    s.active = 0;
    return false;
  }
  s.iter += 1;
  s.rel = sqrt(rr) / s.bnorm;
  if (s.rel < s.best_rel) {
    s.best_rel = s.rel;
    s.best_iter = s.iter;
    s.copy_best = 1;
  } else {
    s.copy_best = 0;
  }
  if (!s.fixed && s.rel <= s.tol) s.active = 0;
  s.beta = rz / s.rho;
  s.rho = rz;
  return true;
}

// Scalar step, then x += alpha p and p = z + beta p (RHS that stepped), in one launch:
// every block folds the partial sums in the same fixed order and derives the same new
// state from st_prev (written by the update, read-only here); block 0 of each RHS
// stores it in st, which no block of this kernel reads.  Tx = double: the iterate lives
// in one of two buffers, x and xbest (CgState.xcur); while it is also the
// lowest-residual one (CgState.xbest) the step writes the new iterate to the other
// buffer, else in place, so the best iterate is kept without a copy.  Tx = float: x
// holds the float32 increment of the iterate since its last float64 fold (reliable
// updates), and no best iterate is kept.
template <typename Tx, typename Tp, typename Tz>
__global__ void k_cg_step_next(Tx* __restrict__ x, double* __restrict__ xbest, Tp* __restrict__ p,
                               const Tz* __restrict__ z, CgState* __restrict__ st,
                               const CgState* __restrict__ st_prev,
                               const double* __restrict__ prz, const double* __restrict__ prr,
                               double* __restrict__ history, int hist_stride, int64_t nu,
                               float* __restrict__ p32, int64_t n32, int64_t vs32) {
  const int r = blockIdx.y;
  const double rz = fold_partials(prz, r);
  const double rr = fold_partials(prr, r);
  CgState s = st_prev[r];
  const bool stepped = cg_scalar_step(s, rz, rr);
  int src = 0, dst = 0;
  if constexpr (sizeof(Tx) == sizeof(double)) {
    if (stepped) {
      src = s.xcur;
      dst = s.xcur == s.xbest ? 1 - s.xcur : s.xcur;
      s.xcur = dst;
      if (s.copy_best) s.xbest = dst;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st[r] = s;
    if (stepped && history) history[(int64_t)r * hist_stride + s.iter % hist_stride] = s.rel;
  }
  // p advances on every step taken, also the one on which an RHS stops: a later
  // residual replacement that finds it above tol continues it along this direction
  if (!stepped) return;
  const double alpha = s.alpha, beta = s.beta;
  // source and destination rows of the iterate (the same buffer, or x and xbest)
  const Tx* xs = src ? reinterpret_cast<const Tx*>(xbest) : x;
  Tx* xd = dst ? reinterpret_cast<Tx*>(xbest) : x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nu; i += stride) {
    const int64_t j = (int64_t)r * nu + i;
    const double pj = (double)p[j];
    xd[j] = (Tx)((double)xs[j] + alpha * pj);
    const double pn = (double)z[j] + beta * pj;
    p[j] = (Tp)pn;
    if (p32 && i < n32) p32[(int64_t)r * vs32 + i] = (float)pn;
  }
}

hipError_t launch_cg_step_next(void* x, bool x_f32, double* xbest, void* p, bool p_f32, const void* z, bool z_f32,
                               CgState* st, const CgState* st_prev, const double* partial_rz,
                               const double* partial_rr, double* history, int hist_stride, int64_t nu, int n_rhs,
                               hipStream_t s, float* p32, int64_t n32, int64_t vs32) {
  dim3 g = grid_for(nu);
  g.y = n_rhs;
  if (x_f32 && p_f32 && z_f32)
    hipLaunchKernelGGL((k_cg_step_next<float, float, float>), g, dim3(256), 0, s, (float*)x, xbest, (float*)p,
                       (const float*)z, st, st_prev, partial_rz, partial_rr, history, hist_stride, nu, p32, n32,
                       vs32);
  else if (x_f32)
    return hipErrorInvalidValue;
  else if (p_f32 && z_f32)
    hipLaunchKernelGGL((k_cg_step_next<double, float, float>), g, dim3(256), 0, s, (double*)x, xbest, (float*)p,
                       (const float*)z, st, st_prev, partial_rz, partial_rr, history, hist_stride, nu, p32, n32,
                       vs32);
  else if (z_f32)
    hipLaunchKernelGGL((k_cg_step_next<double, double, float>), g, dim3(256), 0, s, (double*)x, xbest, (double*)p,
                       (const float*)z, st, st_prev, partial_rz, partial_rr, history, hist_stride, nu, p32, n32,
                       vs32);
  else if (!p_f32)
    hipLaunchKernelGGL((k_cg_step_next<double, double, double>), g, dim3(256), 0, s, (double*)x, xbest, (double*)p,
                       (const double*)z, st, st_prev, partial_rz, partial_rr, history, hist_stride, nu, p32, n32,
                       vs32);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int NS>
__global__ void k_apply_precond(const double* __restrict__ minv, const double* __restrict__ r,
                                double* __restrict__ z, int64_t n_obs, int64_t vs,
                                const double* __restrict__ minv_t, int64_t n_tail, int n_rhs) {
  constexpr int NM = NS == 1 ? 1 : 6;
  const int64_t per = n_obs + n_tail;
  const int64_t n = per * n_rhs;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int64_t rr_ = i / per, o = i % per;
    const int64_t base = rr_ * vs;
    if (o >= n_obs) {   // template amplitude
      const int64_t b = base + n_obs * NS + (o - n_obs);
      z[b] = minv_t[o - n_obs] * r[b];
      continue;
    }
    double rr[NS], zz[NS];
#pragma unroll
    for (int c = 0; c < NS; ++c) rr[c] = r[base + o * NS + c];
    precond_apply<NS>(minv + o * NM, rr, zz);
#pragma unroll
    for (int c = 0; c < NS; ++c) z[base + o * NS + c] = zz[c];
  }
}

hipError_t launch_apply_precond(int ns, const double* minv, const double* r, double* z,
                                int64_t n_obs, int64_t vs, const double* minv_t, int64_t n_tail,
                                int n_rhs, hipStream_t s) {
  const dim3 g = grid_for((n_obs + n_tail) * n_rhs);
  if (ns == 1) hipLaunchKernelGGL(k_apply_precond<1>, g, dim3(256), 0, s, minv, r, z, n_obs, vs, minv_t, n_tail, n_rhs);
  else hipLaunchKernelGGL(k_apply_precond<3>, g, dim3(256), 0, s, minv, r, z, n_obs, vs, minv_t, n_tail, n_rhs);
  return hipGetLastError();
}

__global__ void k_axpby(double* __restrict__ y, const double* __restrict__ x, double a, double b,
                        int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    y[i] = a * x[i] + b * y[i];
}

hipError_t launch_axpby(double* y, const double* x, double a, double b, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpby, grid_for(n), dim3(256), 0, s, y, x, a, b, n);
  return hipGetLastError();
}

__global__ void k_sub(double* __restrict__ out, const double* __restrict__ a,
                      const double* __restrict__ b, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = a[i] - b[i];
}

hipError_t launch_sub(double* out, const double* a, const double* b, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sub, grid_for(n), dim3(256), 0, s, out, a, b, n);
  return hipGetLastError();
}

// x += d, then d = 0
__global__ void k_fold_f32(double* __restrict__ x, float* __restrict__ d, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    x[i] += (double)d[i];
    d[i] = 0.0f;
  }
}

hipError_t launch_fold_f32(double* x, float* d, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold_f32, grid_for(n), dim3(256), 0, s, x, d, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- preconditioner
// kind 0: block (P^T W^-1 P)^-1 with W^-1 = diag(N^-1) = f_b(0) of each sample's interval;
// kind 1: point Jacobi diag(P^T P)^-1;  kind 2: identity.
// A group of G lanes owns a pixel: lanes stride over its samples, the six
// block entries are reduced across the group, and lane 0 inverts in float64.
template <int NS, int G>
__global__ __launch_bounds__(256) void k_precond_build(
    int kind, const int64_t* __restrict__ pix_ptr, const int32_t* __restrict__ perm,
    const float2* __restrict__ w_pm, const int64_t* __restrict__ iv_start, int n_iv,
    const int32_t* __restrict__ iv_hint, int hint_shift, const int32_t* __restrict__ iv_filter,
    const double* __restrict__ lags, int n_c, int64_t n_obs, double* __restrict__ minv,
    int32_t* __restrict__ singular) {
  constexpr int NM = NS == 1 ? 1 : 6;
  constexpr int GPB = 256 / G;
  const int lane = threadIdx.x % G;
  const int64_t stride = (int64_t)gridDim.x * GPB;
  for (int64_t o = (int64_t)blockIdx.x * GPB + threadIdx.x / G; o < n_obs; o += stride) {
    double B[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (kind != 2) {
      for (int64_t k = pix_ptr[o] + lane; k < pix_ptr[o + 1]; k += G) {
        double wgt = 1.0;
        if (kind == 0) {
          const int64_t t = perm[k];
          int b = iv_hint[t >> hint_shift];   // then the last interval with iv_start <= t
          while (b + 1 < n_iv && iv_start[b + 1] <= t) ++b;
          wgt = lags[(int64_t)iv_filter[b] * n_c];
        }
        if (NS == 1) {
          B[0] += wgt;
        } else {
          const float2 sc = w_pm[k];
          const double a0 = 0.5, a1 = 0.5 * (double)sc.x, a2 = 0.5 * (double)sc.y;
          B[0] += wgt * a0 * a0;
          B[1] += wgt * a0 * a1;
          B[2] += wgt * a0 * a2;
          B[3] += wgt * a1 * a1;
          B[4] += wgt * a1 * a2;
          B[5] += wgt * a2 * a2;
        }
      }
#pragma unroll
      for (int c = 0; c < (NS == 1 ? 1 : 6); ++c) B[c] = group_sum<G>(B[c]);
    }
    if (lane != 0) continue;
    double* m = minv + o * NM;
    int32_t bad = 0;
    if (kind == 2) {
      m[0] = 1.0;
      if (NS == 3) { m[1] = 0.0; m[2] = 0.0; m[3] = 1.0; m[4] = 0.0; m[5] = 1.0; }
    } else if (NS == 1) {
      bad = !(B[0] > 0.0);
      m[0] = bad ? 0.0 : 1.0 / B[0];
    } else if (kind == 1) {
      bad = !(B[0] > 0.0 && B[3] > 0.0 && B[5] > 0.0);
      m[0] = bad ? 0.0 : 1.0 / B[0];
      m[3] = bad ? 0.0 : 1.0 / B[3];
      m[5] = bad ? 0.0 : 1.0 / B[5];
      m[1] = m[2] = m[4] = 0.0;
    } else {
      // symmetric 3x3 inverse by cofactors
      const double a = B[0], b = B[1], c = B[2], d = B[3], e = B[4], f = B[5];
      const double c00 = d * f - e * e, c01 = c * e - b * f, c02 = b * e - c * d;
      const double c11 = a * f - c * c, c12 = b * c - a * e, c22 = a * d - b * b;
      const double det = a * c00 + b * c01 + c * c02;
      bad = !(det > 1e-10 * a * d * f) || !isfinite(det);
      const double id = bad ? 0.0 : 1.0 / det;
      m[0] = c00 * id; m[1] = c01 * id; m[2] = c02 * id;
      m[3] = c11 * id; m[4] = c12 * id; m[5] = c22 * id;
    }
    singular[o] = bad;
  }
}

template <int NS>
static hipError_t precond_g(int group, dim3 g, hipStream_t s, int kind, const int64_t* pp,
                            const int32_t* perm, const float2* w, const int64_t* ivs, int n_iv,
                            const int32_t* hint, int hsh, const int32_t* ivf, const double* lags, int n_c,
                            int64_t n_obs, double* minv, int32_t* sing) {
  const dim3 b(256);
  switch (group) {
#define MM_PCB(G) case G: hipLaunchKernelGGL((k_precond_build<NS, G>), g, b, 0, s, kind, pp, perm, w, ivs, n_iv, hint, hsh, ivf, lags, n_c, n_obs, minv, sing); break;
    MM_PCB(4) MM_PCB(8) MM_PCB(16) MM_PCB(32) MM_PCB(64)
#undef MM_PCB
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_precond_build(int ns, int kind, int group, const int64_t* pix_ptr, const int32_t* perm,
                                const float* w_pm, const int64_t* iv_start, int n_iv, const int32_t* iv_hint,
                                int hint_shift, const int32_t* iv_filter, const double* lags, int n_c,
                                int64_t n_obs, double* minv, int32_t* singular, hipStream_t s) {
  if (n_obs == 0) return hipSuccess;
  int64_t nb = (n_obs * group + 255) / 256;
  if (nb > 65536) nb = 65536;
  const dim3 g((unsigned)nb);
  const float2* w = (const float2*)w_pm;
  return ns == 1 ? precond_g<1>(group, g, s, kind, pix_ptr, perm, w, iv_start, n_iv, iv_hint, hint_shift, iv_filter,
                                 lags, n_c, n_obs, minv, singular)
                 : precond_g<3>(group, g, s, kind, pix_ptr, perm, w, iv_start, n_iv, iv_hint, hint_shift, iv_filter,
                                 lags, n_c, n_obs, minv, singular);
}

__global__ __launch_bounds__(256) void k_interval_dots(const double* __restrict__ u,
                                                       const double* __restrict__ v,
                                                       const int64_t* __restrict__ iv_start,
                                                       double* __restrict__ out) {
  __shared__ double sh[256 / 64];
  const int64_t a = iv_start[blockIdx.x], e = iv_start[blockIdx.x + 1];
  double acc = 0.0;
  for (int64_t t = a + threadIdx.x; t < e; t += 256) acc += u[t] * v[t];
  const double sum = block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = sum;
}

hipError_t launch_interval_dots(const double* u, const double* v, const int64_t* iv_start, int n_iv,
                                double* out, hipStream_t s) {
  if (n_iv == 0) return hipSuccess;
  hipLaunchKernelGGL(k_interval_dots, dim3((unsigned)n_iv), dim3(256), 0, s, u, v, iv_start, out);
  return hipGetLastError();
}

// number of nonzero flags, added to *out (an exact integer count, whatever the order)
__global__ __launch_bounds__(256) void k_count_nonzero(const int32_t* __restrict__ flags, int64_t n,
                                                       unsigned long long* __restrict__ out) {
  unsigned int c = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) c += flags[i] != 0 ? 1u : 0u;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0 && c != 0) atomicAdd(out, (unsigned long long)c);
}

hipError_t launch_count_nonzero(const int32_t* flags, int64_t n, unsigned long long* out, hipStream_t s) {
  hipError_t e = hipMemsetAsync(out, 0, sizeof(unsigned long long), s);   // plan time only, never captured
  if (e != hipSuccess || n == 0) return e;
  int64_t nb = (n + 255) / 256;
  if (nb > 2048) nb = 2048;
  hipLaunchKernelGGL(k_count_nonzero, dim3((unsigned)nb), dim3(256), 0, s, flags, n, out);
  return hipGetLastError();
}

}  // namespace mm
