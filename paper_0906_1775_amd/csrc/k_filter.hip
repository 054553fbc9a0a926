// Inverse-noise filter N^-1: lag construction, overlap-save spectra and the
// overlap-save transform kernel (gfx950).
//
// Weighting section of the MADmap paper: N^-1 is block diagonal with a
// banded Toeplitz block per stationary interval, (N^-1)_{t,t'} = f(|t-t'|)
// for |t - t'| < n_c.  A band of half-width n_c is applied exactly by a
// circulant of length n_f on a window that starts n_c samples before the
// first wanted output; each transform yields m = n_f - 2 n_c exact outputs
// (the chunked scheme of eq. FFTcomplexity).
//
// Lags (the paper leaves the construction of f from p(f) open): f is the
// inverse DFT over L_K frequencies nu_j = j f_samp / L_K of 1/p(nu_j),
// p = sigma^2 (1 + (f_knee/nu)^alpha) (Algorithm section), 1/p(0) taken as its
// limit, times the Bartlett taper (1 - tau/n_c).  Only tau < n_c is needed, so
// the L_K-point inverse DFT is split as j = r + R q (R = L_K / n_c'):
//   G_r(tau) = sum_q s_{r + R q} e^{+2 pi i q tau / n_c'}   (R transforms of n_c' points)
//   f~(tau)  = (1/L_K) Re sum_r e^{+2 pi i r tau / L_K} G_r(tau).
#include "fft.hpp"
#include "mm_internal.h"

namespace mm {

// ---------------------------------------------------------------- transform shapes
// (threads, log2 points per thread) of the workgroup transform of 2^LOGN points
template <int LOGN> struct Shape;
template <> struct Shape<6> { static constexpr int NT = 16, LOGE = 2; };
template <> struct Shape<7> { static constexpr int NT = 32, LOGE = 2; };
template <> struct Shape<8> { static constexpr int NT = 64, LOGE = 2; };
template <> struct Shape<9> { static constexpr int NT = 64, LOGE = 3; };
template <> struct Shape<10> { static constexpr int NT = 128, LOGE = 3; };
template <> struct Shape<11> { static constexpr int NT = 256, LOGE = 3; };
template <> struct Shape<12> { static constexpr int NT = 256, LOGE = 4; };
template <> struct Shape<13> { static constexpr int NT = 512, LOGE = 4; };
template <> struct Shape<14> { static constexpr int NT = 1024, LOGE = 4; };

constexpr int kMinLogN = 6;
constexpr int kMaxLogNF32 = 14;   // n_f = 2^15
constexpr int kMaxLogNF64 = 14;   // n_f = 2^15

int ols_max_logn(bool fp64) { return fp64 ? kMaxLogNF64 : kMaxLogNF32; }

// ---------------------------------------------------------------- tables
template <typename T>
__global__ void k_tw2(cx<T>* tw2, int N) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  double s, c;
  sincospi((double)k / (double)N, &s, &c);  // angle pi k / N = 2 pi k / (2N)
  tw2[k] = {(T)c, (T)(-s)};
}

hipError_t launch_tw2_table(void* tw2, int logn, bool fp64, hipStream_t s) {
  const int N = 1 << logn;
  const int nb = (N + 255) / 256;
  if (fp64)
    hipLaunchKernelGGL(k_tw2<double>, dim3(nb), dim3(256), 0, s, (cx<double>*)tw2, N);
  else
    hipLaunchKernelGGL(k_tw2<float>, dim3(nb), dim3(256), 0, s, (cx<float>*)tw2, N);
  return hipGetLastError();
}

// 1/p(nu_j) on the L-point grid, Hermitian-extended: s_j = s_{L-j}
__device__ __forceinline__ double inv_psd(int64_t j, int64_t L, double f_samp, double sigma,
                                          double fknee, double alpha) {
  if (j > L / 2) j = L - j;
  if (j == 0) return fknee > 0.0 ? 0.0 : 1.0 / (sigma * sigma);
  const double nu = (double)j * (f_samp / (double)L);
  return 1.0 / (sigma * sigma * (1.0 + pow(fknee / nu, alpha)));
}

// step 1: grid (R, filters in batch); one n_c'-point transform per (r, filter)
template <int LOGN>
__global__ __launch_bounds__(Shape<LOGN>::NT) void k_lag_step1(
    const double* __restrict__ params, int f0, double f_samp, int64_t L, int n_c,
    const cx<double>* __restrict__ tw2, cx<double>* __restrict__ G) {
  using F = BlockFFT<double, LOGN, Shape<LOGN>::NT, Shape<LOGN>::LOGE>;
  __shared__ __align__(16) char lds[F::LDS_BYTES];
  constexpr int N = F::N, E = F::E;
  const int t = threadIdx.x;
  const int64_t R = L >> LOGN;
  const int64_t r = blockIdx.x;
  const int fl = f0 + blockIdx.y;
  const double sg = params[3 * fl], fk = params[3 * fl + 1], al = params[3 * fl + 2];
  cx<double> v[E];
  constexpr int L0 = F::first_log_fwd(), R0 = 1 << L0;
#pragma unroll
  for (int i = 0; i < E / R0; ++i)
#pragma unroll
    for (int rr = 0; rr < R0; ++rr) {
      const int q = F::template in_index<L0>(t, i, rr);
      v[i * R0 + rr] = {inv_psd(r + R * (int64_t)q, L, f_samp, sg, fk, al), 0.0};
    }
  F::forward(v, lds, tw2, t);
  constexpr int LL = F::last_log_fwd(), RL = 1 << LL;
  cx<double>* out = G + ((int64_t)blockIdx.y * R + r) * n_c;
#pragma unroll
  for (int i = 0; i < E / RL; ++i)
#pragma unroll
    for (int rr = 0; rr < RL; ++rr) {
      const int tau = t + i * F::NT + rr * (N >> LL);
      if (tau < n_c) out[tau] = cconj(v[i * RL + rr]);
    }
}

// step 2: lags[f][tau] = taper * (1/L) Re sum_r e^{2 pi i r tau / L} G_r(tau)
__global__ void k_lag_step2(const cx<double>* __restrict__ G, int f0, int64_t L, int64_t R,
                            int n_c, double* __restrict__ lags) {
  const int tau = blockIdx.x * blockDim.x + threadIdx.x;
  if (tau >= n_c) return;
  const cx<double>* g = G + (int64_t)blockIdx.y * R * n_c + tau;
  double acc = 0.0;
  for (int64_t r = 0; r < R; ++r) {
    const int64_t k = (r * (int64_t)tau) & (L - 1);
    double sn, cs;
    sincospi(2.0 * (double)k / (double)L, &sn, &cs);
    const cx<double> z = g[r * n_c];
    acc += cs * z.re - sn * z.im;
  }
  lags[(int64_t)(f0 + blockIdx.y) * n_c + tau] =
      acc / (double)L * (1.0 - (double)tau / (double)n_c);
}

static int ceil_log2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

size_t lags_scratch_bytes(int n_c, int64_t lag_len, int filters_per_batch) {
  const int logn = ceil_log2(n_c) < kMinLogN ? kMinLogN : ceil_log2(n_c);
  const int64_t R = lag_len >> logn;
  return (size_t)(1 << logn) * 16                                 // twiddles
         + (size_t)filters_per_batch * R * n_c * sizeof(cx<double>);
}

template <int LOGN>
static hipError_t lag_step1(dim3 g, hipStream_t s, const double* params, int f0, double fs,
                            int64_t L, int n_c, const cx<double>* tw2, cx<double>* G) {
  hipLaunchKernelGGL(k_lag_step1<LOGN>, g, dim3(Shape<LOGN>::NT), 0, s, params, f0, fs, L, n_c,
                     tw2, G);
  return hipGetLastError();
}

hipError_t launch_lags(const double* params, int n_filters, double f_samp, int n_c,
                       int64_t lag_len, double* lags, void* scratch, size_t scratch_bytes,
                       hipStream_t s) {
  int logn = ceil_log2(n_c);
  if (logn < kMinLogN) logn = kMinLogN;
  if (logn > kMaxLogNF64) return hipErrorInvalidValue;
  const int64_t R = lag_len >> logn;
  if (R < 2 || (R << logn) != lag_len) return hipErrorInvalidValue;
  cx<double>* tw2 = (cx<double>*)scratch;
  cx<double>* G = (cx<double>*)((char*)scratch + (size_t)(1 << logn) * 16);
  const size_t per_filter = (size_t)R * n_c * sizeof(cx<double>);
  const size_t avail = scratch_bytes - (size_t)(1 << logn) * 16;
  int batch = (int)(avail / per_filter);
  if (batch < 1) return hipErrorInvalidValue;
  hipError_t e = launch_tw2_table(tw2, logn, true, s);
  if (e != hipSuccess) return e;
  for (int f0 = 0; f0 < n_filters; f0 += batch) {
    const int nb = (n_filters - f0) < batch ? (n_filters - f0) : batch;
    const dim3 g1((unsigned)R, (unsigned)nb);
    switch (logn) {
      case 6: e = lag_step1<6>(g1, s, params, f0, f_samp, lag_len, n_c, tw2, G); break;
      case 7: e = lag_step1<7>(g1, s, params, f0, f_samp, lag_len, n_c, tw2, G); break;
      case 8: e = lag_step1<8>(g1, s, params, f0, f_samp, lag_len, n_c, tw2, G); break;
      case 9: e = lag_step1<9>(g1, s, params, f0, f_samp, lag_len, n_c, tw2, G); break;
      case 10: e = lag_step1<10>(g1, s, params, f0, f_samp, lag_len, n_c, tw2, G); break;
      case 11: e = lag_step1<11>(g1, s, params, f0, f_samp, lag_len, n_c, tw2, G); break;
      case 12: e = lag_step1<12>(g1, s, params, f0, f_samp, lag_len, n_c, tw2, G); break;
      case 13: e = lag_step1<13>(g1, s, params, f0, f_samp, lag_len, n_c, tw2, G); break;
      case 14: e = lag_step1<14>(g1, s, params, f0, f_samp, lag_len, n_c, tw2, G); break;
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    const dim3 g2((unsigned)((n_c + 255) / 256), (unsigned)nb);
    hipLaunchKernelGGL(k_lag_step2, g2, dim3(256), 0, s, G, f0, lag_len, R, n_c, lags);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------- spectra
__global__ void k_cos_table(double* ctab, int nf) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < nf) ctab[j] = cospi(2.0 * (double)j / (double)nf);
}

// spec[f][k] = F_k / (4N), F_k = f(0) + 2 sum_{tau=1}^{n_c-1} f(tau) cos(2 pi k tau / n_f), k <= N
template <typename T>
__global__ void k_spectrum(const double* __restrict__ lags, int n_c, int N,
                           const double* __restrict__ ctab, T* __restrict__ spec) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > N) return;
  const double* f = lags + (int64_t)blockIdx.y * n_c;
  const int nf = 2 * N;
  double acc = 0.0;
  int idx = 0;
  for (int tau = 1; tau < n_c; ++tau) {
    idx += k;
    if (idx >= nf) idx -= nf;
    acc += f[tau] * ctab[idx];
  }
  const double F = f[0] + 2.0 * acc;
  spec[(int64_t)blockIdx.y * (N + 1) + k] = (T)(F / (4.0 * (double)N));
}

hipError_t launch_spectra(const double* lags, int n_filters, int n_c, int logn, bool fp64,
                          void* spec, double* ctab, hipStream_t s) {
  const int N = 1 << logn, nf = 2 * N;
  hipLaunchKernelGGL(k_cos_table, dim3((nf + 255) / 256), dim3(256), 0, s, ctab, nf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 g((unsigned)((N + 1 + 255) / 256), (unsigned)n_filters);
  if (fp64)
    hipLaunchKernelGGL(k_spectrum<double>, g, dim3(256), 0, s, lags, n_c, N, ctab, (double*)spec);
  else
    hipLaunchKernelGGL(k_spectrum<float>, g, dim3(256), 0, s, lags, n_c, N, ctab, (float*)spec);
  return hipGetLastError();
}

// ---------------------------------------------------------------- overlap-save transform
// One workgroup per (chunk, RHS).  The n_f = 2N real window u is packed as N
// complex points z_k = u_{2k} + i u_{2k+1}; after the forward transform Z, the
// spectrum of u is X_k = E_k + W^k O_k, X_{k+N} = E_k - W^k O_k with
// E = (Z_k + conj Z_{N-k})/2, O = (Z_k - conj Z_{N-k})/(2i), W = e^{-2 pi i/(2N)}.
// Multiplying by the filter symbol F and folding back gives the packed
// spectrum of the output, Z'_k = (Y_k + Y_{k+N})/2 + i W^{-k} (Y_k - Y_{k+N})/2,
// Y = F X.  The table spec holds F/(4N), which absorbs both halvings and the
// 1/N of the inverse transform; the inverse is conj(FFT(conj Z')).
template <typename T, typename Tin, int LOGN>
__global__ __launch_bounds__(Shape<LOGN>::NT) void k_ols(
    const Tin* __restrict__ yin, T* __restrict__ yout, const OlsChunk* __restrict__ chunks,
    const T* __restrict__ spec, const cx<T>* __restrict__ tw2, int64_t n_t, int n_c, int m) {
  using F = BlockFFT<T, LOGN, Shape<LOGN>::NT, Shape<LOGN>::LOGE>;
  __shared__ __align__(16) char lds[F::LDS_BYTES];
  constexpr int N = F::N, E = F::E, NT = F::NT;
  const int t = threadIdx.x;
  const OlsChunk ch = chunks[blockIdx.x];
  const int64_t roff = (int64_t)blockIdx.y * n_t;
  const int64_t s0 = ch.out_start - n_c;
  const int64_t lo = ch.iv_lo, hi = ch.iv_hi;
  const Tin* __restrict__ src = yin + roff;

  cx<T> v[E];
  constexpr int L0 = F::first_log_fwd(), R0 = 1 << L0;
#pragma unroll
  for (int i = 0; i < E / R0; ++i)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int k = F::template in_index<L0>(t, i, r);
      const int64_t j = s0 + 2 * (int64_t)k;
      const T a = (j >= lo && j < hi) ? (T)src[j] : (T)0;
      const T b = (j + 1 >= lo && j + 1 < hi) ? (T)src[j + 1] : (T)0;
      v[i * R0 + r] = {a, b};
    }

  F::forward(v, lds, tw2, t);

  // pair Z_k with Z_{N-k} through LDS and apply the filter symbol
  constexpr int LL = F::last_log_fwd(), RL = 1 << LL, NBL = E / RL;
  const T* __restrict__ S = spec + (int64_t)ch.filter * (N + 1);
  auto symbol = [&](int k, cx<T> A, cx<T> partner) -> cx<T> {
    const cx<T> B = cconj(partner);
    const cx<T> Ev = cadd(A, B);
    const cx<T> D = csub(A, B);
    const cx<T> O = {D.im, -D.re};            // -i (A - B)
    const cx<T> W = tw2[k];                    // e^{-2 pi i k / (2N)}
    const cx<T> WO = cmul(W, O);
    const T sa = S[k], sb = S[N - k];
    const cx<T> Y = cscale(cadd(Ev, WO), sa);
    const cx<T> Yp = cscale(csub(Ev, WO), sb);
    const cx<T> sum = cadd(Y, Yp);
    const cx<T> dif = csub(Y, Yp);
    const cx<T> Wd = cmul(cconj(W), dif);      // W^{-k} (Y - Y')
    return {sum.re - Wd.im, -(sum.im + Wd.re)};  // conj(sum + i Wd)
  };
  if constexpr (!F::SPLIT) {
    cx<T>* l = reinterpret_cast<cx<T>*>(lds);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NBL; ++i)
#pragma unroll
      for (int r = 0; r < RL; ++r) l[F::cpad(t + i * NT + r * (N >> LL))] = v[i * RL + r];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NBL; ++i)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int k = t + i * NT + r * (N >> LL);
        v[i * RL + r] = symbol(k, v[i * RL + r], l[F::cpad((N - k) & (N - 1))]);
      }
  } else {
    T* l = reinterpret_cast<T*>(lds);
    T pre[E];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NBL; ++i)
#pragma unroll
      for (int r = 0; r < RL; ++r) l[F::spad(t + i * NT + r * (N >> LL))] = v[i * RL + r].re;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NBL; ++i)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int k = t + i * NT + r * (N >> LL);
        pre[i * RL + r] = l[F::spad((N - k) & (N - 1))];
      }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NBL; ++i)
#pragma unroll
      for (int r = 0; r < RL; ++r) l[F::spad(t + i * NT + r * (N >> LL))] = v[i * RL + r].im;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NBL; ++i)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int k = t + i * NT + r * (N >> LL);
        const cx<T> partner = {pre[i * RL + r], l[F::spad((N - k) & (N - 1))]};
        v[i * RL + r] = symbol(k, v[i * RL + r], partner);
      }
  }

  F::forward_rev(v, lds, tw2, t);

  constexpr int LZ = F::last_log_rev(), RZ = 1 << LZ;
  T* __restrict__ dst = yout + roff;
#pragma unroll
  for (int i = 0; i < E / RZ; ++i)
#pragma unroll
    for (int r = 0; r < RZ; ++r) {
      const int j = t + i * NT + r * (N >> LZ);
      const int pos = 2 * j;
      const cx<T> z = v[i * RZ + r];
      if (pos >= n_c && pos < n_c + m && s0 + pos < hi) dst[s0 + pos] = z.re;
      if (pos + 1 >= n_c && pos + 1 < n_c + m && s0 + pos + 1 < hi) dst[s0 + pos + 1] = -z.im;
    }
}

template <typename T, typename Tin, int LOGN>
static hipError_t ols_launch(const void* y_in, void* y_out, const OlsChunk* chunks, int n_chunks,
                             const void* spec, const void* tw2, int64_t n_t, int n_c, int m,
                             int n_rhs, hipStream_t s) {
  hipLaunchKernelGGL((k_ols<T, Tin, LOGN>), dim3((unsigned)n_chunks, (unsigned)n_rhs),
                     dim3(Shape<LOGN>::NT), 0, s, (const Tin*)y_in, (T*)y_out, chunks,
                     (const T*)spec, (const cx<T>*)tw2, n_t, n_c, m);
  return hipGetLastError();
}

template <typename T, typename Tin>
static hipError_t ols_dispatch(int logn, const void* y_in, void* y_out, const OlsChunk* chunks,
                               int n_chunks, const void* spec, const void* tw2, int64_t n_t,
                               int n_c, int m, int n_rhs, hipStream_t s) {
#define MM_OLS_CASE(L) \
  case L: return ols_launch<T, Tin, L>(y_in, y_out, chunks, n_chunks, spec, tw2, n_t, n_c, m, n_rhs, s);
  switch (logn) {
    MM_OLS_CASE(6)
    MM_OLS_CASE(7)
    MM_OLS_CASE(8)
    MM_OLS_CASE(9)
    MM_OLS_CASE(10)
    MM_OLS_CASE(11)
    MM_OLS_CASE(12)
    MM_OLS_CASE(13)
    MM_OLS_CASE(14)
    default: break;
  }
#undef MM_OLS_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_ols(bool fp64, bool in_f64, int logn, const void* y_in, void* y_out,
                      const OlsChunk* chunks, int n_chunks, const void* spec, const void* tw2,
                      int64_t n_t, int n_c, int m, int n_rhs, hipStream_t s) {
  if (n_chunks == 0 || n_rhs == 0) return hipSuccess;
  if (fp64) {
    return in_f64 ? ols_dispatch<double, double>(logn, y_in, y_out, chunks, n_chunks, spec, tw2,
                                                 n_t, n_c, m, n_rhs, s)
                  : ols_dispatch<double, float>(logn, y_in, y_out, chunks, n_chunks, spec, tw2,
                                                n_t, n_c, m, n_rhs, s);
  }
  return in_f64 ? ols_dispatch<float, double>(logn, y_in, y_out, chunks, n_chunks, spec, tw2, n_t,
                                              n_c, m, n_rhs, s)
                : ols_dispatch<float, float>(logn, y_in, y_out, chunks, n_chunks, spec, tw2, n_t,
                                             n_c, m, n_rhs, s);
}

}  // namespace mm
