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
// and the log2 of the largest radix
template <int LOGN> struct Shape;
template <> struct Shape<6> { static constexpr int NT = 16, LOGE = 2, LOGR = 2; };
template <> struct Shape<7> { static constexpr int NT = 32, LOGE = 2, LOGR = 2; };
template <> struct Shape<8> { static constexpr int NT = 64, LOGE = 2, LOGR = 2; };
template <> struct Shape<9> { static constexpr int NT = 64, LOGE = 3, LOGR = 3; };
template <> struct Shape<10> { static constexpr int NT = 128, LOGE = 3, LOGR = 3; };
template <> struct Shape<11> { static constexpr int NT = 256, LOGE = 3, LOGR = 3; };
template <> struct Shape<12> { static constexpr int NT = 256, LOGE = 4, LOGR = 4; };
template <> struct Shape<13> { static constexpr int NT = 512, LOGE = 4, LOGR = 4; };
template <> struct Shape<14> { static constexpr int NT = 1024, LOGE = 4, LOGR = 4; };
template <> struct Shape<15> { static constexpr int NT = 1024, LOGE = 5, LOGR = 4; };

constexpr int kMinLogN = 6;
constexpr int kMaxLogNF32 = 15;   // n_f = 2^16
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

// Workgroup shapes of the overlap-save transform; the autotuner may pick any
// shape that exists for a length and precision.  Variant 0 is Shape<LOGN>.
// Variant 1 uses half the threads with twice the points each and radix-32
// passes: a 2^14-point transform then takes three register passes and two LDS
// exchanges instead of four and three, at 2 wavefronts per SIMD instead of 4.
// Variant 2 is that thread count with radix-16 passes, two butterflies per
// thread and the paired layout, so the conjugate pairs of the real-to-complex
// step meet in registers.  Variant 3 is variant 2 with the LDS exchanges split
// into real and imaginary halves (68 KB) and at most 128 VGPRs, so that two
// workgroups share a CU and one's global loads and stores overlap the other's
// arithmetic.  Variant 4 is 256 threads x 64 points with radix-32 passes, split
// and two per CU.  Variant 5 is 1024 threads x 16 points with radix-8 passes
// and the paired layout (the fastest 2^14-point shape measured in float32);
// variant 6 is variant 5 split, two per CU; variant 7 is 512 threads
// x 32 points with radix-8 passes, paired; variant 8 is variant 5 with half
// exchanges (the lower half of the index space, then the upper half, through an
// LDS buffer of N/2 points), two per CU at 64 VGPRs; variant 9 is the four-step
// transform with wavefront-private inner stages (k_ols_wave.hip; its "pass twiddles"
// are that kernel's tables and its symbol is read in row order).  In float64 the 512-thread shapes
// (variants 2 and 7) have twice the registers per thread, and variant 2 is the
// fastest there.  BPC: workgroups per CU the register budget is sized for.
template <int NT_, int LOGE_, int LOGR_, bool SPLIT_ = false, bool PAIRED_ = false, int BPC_ = 1,
          bool HALF_ = false>
struct OlsCfg {
  static constexpr int NT = NT_, LOGE = LOGE_, LOGR = LOGR_, BPC = BPC_;
  static constexpr bool SPLIT = SPLIT_, PAIRED = PAIRED_, HALF = HALF_;
  // minimum wavefronts per SIMD asked of the register allocator
  static constexpr int WPE = (BPC_ * NT_ / 256) > 1 ? (BPC_ * NT_ / 256) : 1;
};
template <int LOGN, int V> struct OlsShape : OlsCfg<Shape<LOGN>::NT, Shape<LOGN>::LOGE, Shape<LOGN>::LOGR> {};
template <> struct OlsShape<15, 0> : OlsCfg<1024, 5, 4, false, true> {};
template <> struct OlsShape<13, 1> : OlsCfg<256, 5, 5> {};
template <> struct OlsShape<14, 1> : OlsCfg<512, 5, 5> {};
template <> struct OlsShape<14, 2> : OlsCfg<512, 5, 4, false, true> {};
template <> struct OlsShape<14, 3> : OlsCfg<512, 5, 4, true, true, 2> {};
template <> struct OlsShape<14, 4> : OlsCfg<256, 6, 5, true, true, 2> {};
template <> struct OlsShape<14, 5> : OlsCfg<1024, 4, 3, false, true> {};
template <> struct OlsShape<14, 6> : OlsCfg<1024, 4, 3, true, true, 2> {};
template <> struct OlsShape<14, 7> : OlsCfg<512, 5, 3, false, true> {};
template <> struct OlsShape<14, 8> : OlsCfg<1024, 4, 3, false, true, 2, true> {};
template <> struct OlsShape<15, 1> : OlsCfg<512, 6, 5, false, true> {};
template <> struct OlsShape<15, 2> : OlsCfg<1024, 5, 3, false, true> {};

bool ols_variant_exists(int logn, bool fp64, int v) {
  if (v == 0) return logn >= kMinLogN && logn <= ols_max_logn(fp64);
  if (v == 9) return ols_wave_exists(logn, fp64);
  if (v == 5 || v == 7 || (v == 2 && logn == 14)) return logn == 14;
  if (fp64) return false;
  return (v == 1 && (logn == 13 || logn == 14 || logn == 15)) || ((v >= 2 && v <= 6) && logn == 14) ||
         (v == 8 && logn == 14) ||
         (v == 2 && logn == 15);
}

template <typename T, int LOGN, int V = 0>
using ShapeFFT = BlockFFT<T, LOGN, OlsShape<LOGN, V>::NT, OlsShape<LOGN, V>::LOGE, OlsShape<LOGN, V>::LOGR,
                          OlsShape<LOGN, V>::SPLIT, OlsShape<LOGN, V>::PAIRED, OlsShape<LOGN, V>::HALF>;

// per-pass twiddle rows: entry (j, r) of pass p = exp(-2 pi i j r / (Ns R))
template <typename T, int LOGN, int V>
__global__ void k_pass_tw(cx<T>* tab) {
  using F = ShapeFFT<T, LOGN, V>;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= F::tw_total()) return;
  for (int sq = 0; sq < 2; ++sq) {
    const bool fwd = sq == 0;
    for (int p = 0; p < F::NP; ++p) {
      const int o = F::tw_offset(fwd, p), c = F::tw_count(fwd, p);
      if (e >= o && e < o + c) {
        const int lr = F::log_radix(fwd, p), ls = F::log_span(fwd, p);
        const int j = (e - o) >> lr, r = (e - o) & ((1 << lr) - 1);
        const double frac = (double)((int64_t)j * r) / (double)(1 << (lr + ls));
        double sn, cs;
        sincospi(2.0 * frac, &sn, &cs);
        tab[e] = {(T)cs, (T)(-sn)};
        return;
      }
    }
  }
}

template <typename T, int LOGN, int V = 0>
static int pass_tw_total_t() { return ShapeFFT<T, LOGN, V>::tw_total(); }

int pass_twiddle_count(int logn, bool fp64, int variant) {
  if (!ols_variant_exists(logn, fp64, variant)) return -1;
  if (variant == 9) return ols_wave_table_count(logn);
  if (variant == 1)
    return logn == 13 ? pass_tw_total_t<float, 13, 1>()
                      : (logn == 14 ? pass_tw_total_t<float, 14, 1>() : pass_tw_total_t<float, 15, 1>());
  if (variant == 2 && fp64) return pass_tw_total_t<double, 14, 2>();
  if (variant == 2) return logn == 14 ? pass_tw_total_t<float, 14, 2>() : pass_tw_total_t<float, 15, 2>();
  if (variant == 7) return fp64 ? pass_tw_total_t<double, 14, 7>() : pass_tw_total_t<float, 14, 7>();
  if (variant == 3) return pass_tw_total_t<float, 14, 3>();
  if (variant == 4) return pass_tw_total_t<float, 14, 4>();
  if (variant == 5) return fp64 ? pass_tw_total_t<double, 14, 5>() : pass_tw_total_t<float, 14, 5>();
  if (variant == 6) return pass_tw_total_t<float, 14, 6>();
  if (variant == 8) return pass_tw_total_t<float, 14, 8>();
#define MM_PTC(L) case L: return fp64 ? pass_tw_total_t<double, L>() : pass_tw_total_t<float, L>();
  switch (logn) {
    MM_PTC(6) MM_PTC(7) MM_PTC(8) MM_PTC(9) MM_PTC(10) MM_PTC(11) MM_PTC(12) MM_PTC(13) MM_PTC(14)
    case 15: return fp64 ? -1 : pass_tw_total_t<float, 15>();
    default: return -1;
  }
#undef MM_PTC
}

template <typename T, int LOGN, int V = 0>
static hipError_t pass_tw_launch(void* tab, hipStream_t s) {
  const int n = ShapeFFT<T, LOGN, V>::tw_total();
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_pass_tw<T, LOGN, V>), dim3((n + 255) / 256), dim3(256), 0, s, (cx<T>*)tab);
  return hipGetLastError();
}

hipError_t launch_pass_twiddles(void* tab, int logn, bool fp64, hipStream_t s, int variant) {
  if (!ols_variant_exists(logn, fp64, variant)) return hipErrorInvalidValue;
  if (variant == 9) return launch_wave_tables(logn, tab, s);
  if (variant == 1)
    return logn == 13 ? pass_tw_launch<float, 13, 1>(tab, s)
                      : (logn == 14 ? pass_tw_launch<float, 14, 1>(tab, s) : pass_tw_launch<float, 15, 1>(tab, s));
  if (variant == 2 && fp64) return pass_tw_launch<double, 14, 2>(tab, s);
  if (variant == 2) return logn == 14 ? pass_tw_launch<float, 14, 2>(tab, s) : pass_tw_launch<float, 15, 2>(tab, s);
  if (variant == 7) return fp64 ? pass_tw_launch<double, 14, 7>(tab, s) : pass_tw_launch<float, 14, 7>(tab, s);
  if (variant == 3) return pass_tw_launch<float, 14, 3>(tab, s);
  if (variant == 4) return pass_tw_launch<float, 14, 4>(tab, s);
  if (variant == 5) return fp64 ? pass_tw_launch<double, 14, 5>(tab, s) : pass_tw_launch<float, 14, 5>(tab, s);
  if (variant == 6) return pass_tw_launch<float, 14, 6>(tab, s);
  if (variant == 8) return pass_tw_launch<float, 14, 8>(tab, s);
#define MM_PTL(L) case L: return fp64 ? pass_tw_launch<double, L>(tab, s) : pass_tw_launch<float, L>(tab, s);
  switch (logn) {
    MM_PTL(6) MM_PTL(7) MM_PTL(8) MM_PTL(9) MM_PTL(10) MM_PTL(11) MM_PTL(12) MM_PTL(13) MM_PTL(14)
    case 15: return fp64 ? hipErrorInvalidValue : pass_tw_launch<float, 15>(tab, s);
    default: return hipErrorInvalidValue;
  }
#undef MM_PTL
}

// 1/p(nu_j) on the L-point grid, Hermitian-extended: s_j = s_{L-j}; mode 1-3
// give its derivative with respect to sigma, f_knee, alpha.  With
// x = (f_knee/nu)^alpha:  ds/dsigma = -2 s/sigma,  ds/df_knee = -s^2 sigma^2 alpha x/f_knee,
// ds/dalpha = -s^2 sigma^2 x ln(f_knee/nu); the nu = 0 value (0 or 1/sigma^2)
// does not depend on f_knee or alpha.
__device__ __forceinline__ double inv_psd(int64_t j, int64_t L, double f_samp, double sigma,
                                          double fknee, double alpha, int mode) {
  if (j > L / 2) j = L - j;
  if (j == 0) {
    const double s0 = fknee > 0.0 ? 0.0 : 1.0 / (sigma * sigma);
    return mode == 0 ? s0 : (mode == 1 ? -2.0 * s0 / sigma : 0.0);
  }
  const double nu = (double)j * (f_samp / (double)L);
  const double x = pow(fknee / nu, alpha);
  const double s = 1.0 / (sigma * sigma * (1.0 + x));
  switch (mode) {
    case 0: return s;
    case 1: return -2.0 * s / sigma;
    case 2: return fknee > 0.0 ? -s * s * sigma * sigma * alpha * x / fknee : 0.0;
    default: return fknee > 0.0 ? -s * s * sigma * sigma * x * log(fknee / nu) : 0.0;
  }
}

// step 1: grid (R, filters in batch); one n_c'-point transform per (r, filter)
template <int LOGN>
__global__ __launch_bounds__(Shape<LOGN>::NT) void k_lag_step1(
    const double* __restrict__ params, int f0, double f_samp, int64_t L, int n_c,
    const cx<double>* __restrict__ ptw, cx<double>* __restrict__ G, int mode) {
  using F = ShapeFFT<double, LOGN>;
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
      v[i * R0 + rr] = {inv_psd(r + R * (int64_t)q, L, f_samp, sg, fk, al, mode), 0.0};
    }
  F::forward(v, lds, ptw, t);
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

static size_t lag_tw_bytes(int logn) {
  const int n = pass_twiddle_count(logn, true);
  return ((size_t)(n > 0 ? n : 1) * sizeof(cx<double>) + 255) & ~(size_t)255;
}

size_t lags_scratch_bytes(int n_c, int64_t lag_len, int filters_per_batch) {
  const int logn = ceil_log2(n_c) < kMinLogN ? kMinLogN : ceil_log2(n_c);
  const int64_t R = lag_len >> logn;
  return lag_tw_bytes(logn) + (size_t)filters_per_batch * R * n_c * sizeof(cx<double>);
}

template <int LOGN>
static hipError_t lag_step1(dim3 g, hipStream_t s, const double* params, int f0, double fs,
                            int64_t L, int n_c, const cx<double>* ptw, cx<double>* G, int mode) {
  hipLaunchKernelGGL(k_lag_step1<LOGN>, g, dim3(Shape<LOGN>::NT), 0, s, params, f0, fs, L, n_c,
                     ptw, G, mode);
  return hipGetLastError();
}

hipError_t launch_lags(const double* params, int n_filters, double f_samp, int n_c,
                       int64_t lag_len, double* lags, void* scratch, size_t scratch_bytes,
                       hipStream_t s, int mode) {
  int logn = ceil_log2(n_c);
  if (logn < kMinLogN) logn = kMinLogN;
  if (logn > kMaxLogNF64) return hipErrorInvalidValue;
  const int64_t R = lag_len >> logn;
  if (R < 2 || (R << logn) != lag_len) return hipErrorInvalidValue;
  cx<double>* ptw = (cx<double>*)scratch;   // per-pass twiddle tables of the transform
  cx<double>* G = (cx<double>*)((char*)scratch + lag_tw_bytes(logn));
  const size_t per_filter = (size_t)R * n_c * sizeof(cx<double>);
  if (scratch_bytes < lag_tw_bytes(logn) + per_filter) return hipErrorInvalidValue;
  const size_t avail = scratch_bytes - lag_tw_bytes(logn);
  const size_t fit = avail / per_filter;
  const int batch = (int)(fit < 65535 ? fit : 65535);   // filters per launch (grid y)
  hipError_t e = launch_pass_twiddles(ptw, logn, true, s);
  if (e != hipSuccess) return e;
  for (int f0 = 0; f0 < n_filters; f0 += batch) {
    const int nb = (n_filters - f0) < batch ? (n_filters - f0) : batch;
    const dim3 g1((unsigned)R, (unsigned)nb);
    switch (logn) {
      case 6: e = lag_step1<6>(g1, s, params, f0, f_samp, lag_len, n_c, ptw, G, mode); break;
      case 7: e = lag_step1<7>(g1, s, params, f0, f_samp, lag_len, n_c, ptw, G, mode); break;
      case 8: e = lag_step1<8>(g1, s, params, f0, f_samp, lag_len, n_c, ptw, G, mode); break;
      case 9: e = lag_step1<9>(g1, s, params, f0, f_samp, lag_len, n_c, ptw, G, mode); break;
      case 10: e = lag_step1<10>(g1, s, params, f0, f_samp, lag_len, n_c, ptw, G, mode); break;
      case 11: e = lag_step1<11>(g1, s, params, f0, f_samp, lag_len, n_c, ptw, G, mode); break;
      case 12: e = lag_step1<12>(g1, s, params, f0, f_samp, lag_len, n_c, ptw, G, mode); break;
      case 13: e = lag_step1<13>(g1, s, params, f0, f_samp, lag_len, n_c, ptw, G, mode); break;
      case 14: e = lag_step1<14>(g1, s, params, f0, f_samp, lag_len, n_c, ptw, G, mode); break;
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

// ---------------------------------------------------------------- pairing helper
// After a forward transform the thread holds Z_k at k = t + i NT + r N/R_last.
// For each of its points, call fn(k, Z_k, Z_{N-k}) -> new value of the point,
// with Z_{N-k} fetched from the owner thread through LDS.
template <typename F, typename T, typename Fn>
__device__ __forceinline__ void with_partner(cx<T>* v, void* lds, int t, Fn fn) {
  constexpr int N = F::N, E = F::E, NT = F::NT;
  constexpr int LL = F::last_log_fwd(), RL = 1 << LL, NBL = E / RL;
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
        v[i * RL + r] = fn(k, v[i * RL + r], l[F::cpad((N - k) & (N - 1))]);
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
        v[i * RL + r] = fn(k, v[i * RL + r], partner);
      }
  }
}

// Paired shapes: after the forward transform the thread already holds Z_{N-k}
// beside each of its Z_k (fft.hpp, paired layout).  fn(k, Z_k, Z_{N-k}, out_k,
// out_{N-k}) replaces both members of a pair.  With NB butterflies per thread,
// element (i, r) of thread t > 0 pairs with (i ^ 1, R - 1 - r); thread 0 owns the
// butterflies i NT: (0, r) pairs with (0, R - r) (k = 0 and k = N/2 are their
// own partners, and then only out_k is kept) and (i, r) with (NB - i, R - 1 - r).
template <typename F, typename T, typename Fn>
__device__ __forceinline__ void with_partner_paired(cx<T>* v, int t, Fn fn) {
  constexpr int N = F::N, R = 1 << F::last_log_fwd(), NB = F::E / R;
  static_assert(F::PAIRED && NB % 2 == 0, "paired layout expected");
  if (t != 0) {
#pragma unroll
    for (int q = 0; q < NB / 2; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r)
        fn(F::fwd_out_index(t, 2 * q, r), v[2 * q * R + r], v[(2 * q + 1) * R + R - 1 - r]);
  } else {
#pragma unroll
    for (int r = 0; r <= R / 2; ++r) {
      if (r == 0 || r == R / 2) {
        cx<T> self = v[r];
        fn(F::fwd_out_index(0, 0, r), v[r], self);
      } else {
        fn(F::fwd_out_index(0, 0, r), v[r], v[R - r]);
      }
    }
#pragma unroll
    for (int i = 1; i < NB / 2; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r) fn(F::fwd_out_index(0, i, r), v[i * R + r], v[(NB - i) * R + R - 1 - r]);
#pragma unroll
    for (int r = 0; r < R / 2; ++r)
      fn(F::fwd_out_index(0, NB / 2, r), v[(NB / 2) * R + r], v[(NB / 2) * R + R - 1 - r]);
  }
}

// ---------------------------------------------------------------- spectra
// Symbol of the circulant that embeds one filter's band:
//   F_k = f(0) + 2 sum_{tau=1}^{n_c-1} f(tau) cos(2 pi k tau / n_f),  k = 0 .. N,
// i.e. the DFT of the real, even first column c (c_i = f(|i|) circularly).  c is
// packed as N complex points, transformed in float64 by one workgroup, and the
// real spectrum recovered with X_k = E_k + W^k O_k (X_N = E_0 - O_0).  The
// table keeps F/(4N) in the filter's working precision.
template <typename T, int LOGN>
__global__ __launch_bounds__(Shape<LOGN>::NT) void k_spectrum_fft(
    const double* __restrict__ lags, int n_c, T* __restrict__ spec,
    const cx<double>* __restrict__ ptw, const cx<double>* __restrict__ tw2) {
  using F = ShapeFFT<double, LOGN>;
  __shared__ __align__(16) char lds[F::LDS_BYTES];
  constexpr int N = F::N, E = F::E;
  const int nf = 2 * N;
  const int t = threadIdx.x;
  const double* __restrict__ f = lags + (int64_t)blockIdx.x * n_c;
  T* __restrict__ out = spec + (int64_t)blockIdx.x * (N + 1);
  auto col = [&](int i) -> double {
    if (i < n_c) return f[i];
    const int j = nf - i;
    return j < n_c ? f[j] : 0.0;
  };
  cx<double> v[E];
  constexpr int L0 = F::first_log_fwd(), R0 = 1 << L0;
#pragma unroll
  for (int i = 0; i < E / R0; ++i)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int k = F::template in_index<L0>(t, i, r);
      v[i * R0 + r] = {col(2 * k), col(2 * k + 1)};
    }
  F::forward(v, lds, ptw, t);
  const double scale = 1.0 / (4.0 * (double)N);
  with_partner<F>(v, lds, t, [&](int k, cx<double> A, cx<double> Bp) {
    const cx<double> B = cconj(Bp);
    const cx<double> Ev = cadd(A, B);                       // 2 E_k
    const cx<double> D = csub(A, B);
    const cx<double> O = {D.im, -D.re};                     // 2 O_k
    const cx<double> X = cadd(Ev, cmul(tw2[k], O));         // 2 X_k
    out[k] = (T)(0.5 * X.re * scale);
    if (k == 0) out[N] = (T)(0.5 * (Ev.re - O.re) * scale);
    return A;
  });
}

// Direct-sum form of the same symbol, for transform lengths beyond the largest
// float64 workgroup transform.  One thread takes k and N - k together: since
// cos(2 pi (N - k) tau / n_f) = (-1)^tau cos(2 pi k tau / n_f), F_k = f(0) + 2 (E + O)
// and F_(N-k) = f(0) + 2 (E - O), E and O the sums over even and odd tau >= 1.  The
// cosines are the real parts of z_tau = exp(2 pi i k tau / n_f), advanced by one
// complex rotation per tau.  A run of kDirectRun steps starts from z at its first tau,
// which advances by one rotation by w^kDirectRun per run and is restarted every
// kDirectRestart runs from a float64 table of cos(2 pi j / n_f), j < n_f (indexed by
// (k tau) mod n_f; the sine is the entry a quarter period earlier): rounding grows over
// at most kDirectRun + kDirectRestart rotations, and a lane reads the table once per
// kDirectRun * kDirectRestart steps (its reads scatter over the table, one cache line each).
constexpr int kDirectRun = 16;
constexpr int kDirectRestart = 16;

__global__ void k_cos_table(double* ctab, int nf) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < nf) ctab[j] = cospi(2.0 * (double)j / (double)nf);
}

template <typename T>
__global__ void k_spectrum_direct(const double* __restrict__ lags, int n_c, int N,
                                  const double* __restrict__ ctab, T* __restrict__ spec) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;   // 0 .. N/2
  if (k > N / 2) return;
  const double* __restrict__ f = lags + (int64_t)blockIdx.y * n_c;
  const int64_t mask = 2 * (int64_t)N - 1, quarter = N / 2;
  auto unit = [&](int64_t j) -> cx<double> {   // (cos, sin) of 2 pi j / n_f
    j &= mask;
    return {ctab[j], ctab[(j - quarter) & mask]};
  };
  const cx<double> w = unit(k);
  const cx<double> w_run = unit((int64_t)k * kDirectRun);
  double ev = 0.0, od = 0.0;
  cx<double> z0 = {1.0, 0.0};
  for (int t0 = 0, run = 0; t0 < n_c; t0 += kDirectRun, ++run) {
    if (run % kDirectRestart == 0) z0 = unit((int64_t)k * t0);
    cx<double> z = z0;
    z0 = cmul(z0, w_run);
#pragma unroll
    for (int i = 0; i < kDirectRun; i += 2) {
      const int tau = t0 + i;   // even
      if (tau >= n_c) break;
      if (tau > 0) ev = fma(f[tau], z.re, ev);
      z = cmul(z, w);
      if (tau + 1 >= n_c) break;
      od = fma(f[tau + 1], z.re, od);
      z = cmul(z, w);
    }
  }
  const double scale = 1.0 / (4.0 * (double)N);
  T* __restrict__ out = spec + (int64_t)blockIdx.y * (N + 1);
  out[k] = (T)((f[0] + 2.0 * (ev + od)) * scale);
  if (N - k != k) out[N - k] = (T)((f[0] + 2.0 * (ev - od)) * scale);
}

template <typename T, int LOGN>
static hipError_t spectrum_launch(const double* lags, int n_filters, int n_c, void* spec,
                                  const void* ptw, const void* tw2, hipStream_t s) {
  hipLaunchKernelGGL((k_spectrum_fft<T, LOGN>), dim3((unsigned)n_filters), dim3(Shape<LOGN>::NT), 0, s,
                     lags, n_c, (T*)spec, (const cx<double>*)ptw, (const cx<double>*)tw2);
  return hipGetLastError();
}

size_t spectra_scratch_bytes(int logn) {
  if (logn > kMaxLogNF64) return (size_t)(2 << logn) * sizeof(double) + 256;   // cosine table
  const int n = pass_twiddle_count(logn, true);
  return (size_t)(n > 0 ? n : 1) * sizeof(cx<double>) + (size_t)(1 << logn) * sizeof(cx<double>) + 256;
}

hipError_t launch_spectra(const double* lags, int n_filters, int n_c, int logn, bool fp64,
                          void* spec, void* scratch, hipStream_t s) {
  if (n_filters == 0) return hipSuccess;
  if (logn > kMaxLogNF64) {
    const int N = 1 << logn, nf = 2 * N;
    double* ctab = (double*)scratch;
    hipLaunchKernelGGL(k_cos_table, dim3((nf + 255) / 256), dim3(256), 0, s, ctab, nf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g((unsigned)((N / 2 + 1 + 255) / 256), (unsigned)n_filters);
    if (fp64)
      hipLaunchKernelGGL(k_spectrum_direct<double>, g, dim3(256), 0, s, lags, n_c, N, ctab, (double*)spec);
    else
      hipLaunchKernelGGL(k_spectrum_direct<float>, g, dim3(256), 0, s, lags, n_c, N, ctab, (float*)spec);
    return hipGetLastError();
  }
  // float64 twiddles for the spectrum transform, whatever the filter's precision
  cx<double>* ptw = (cx<double>*)scratch;
  const int n = pass_twiddle_count(logn, true);
  if (n < 0) return hipErrorInvalidValue;
  cx<double>* tw2 = ptw + (n > 0 ? n : 1);
  hipError_t e = launch_pass_twiddles(ptw, logn, true, s);
  if (e != hipSuccess) return e;
  if ((e = launch_tw2_table(tw2, logn, true, s)) != hipSuccess) return e;
#define MM_SPC(L) \
  case L: return fp64 ? spectrum_launch<double, L>(lags, n_filters, n_c, spec, ptw, tw2, s) \
                      : spectrum_launch<float, L>(lags, n_filters, n_c, spec, ptw, tw2, s);
  switch (logn) {
    MM_SPC(6) MM_SPC(7) MM_SPC(8) MM_SPC(9) MM_SPC(10) MM_SPC(11) MM_SPC(12) MM_SPC(13) MM_SPC(14)
    default: return hipErrorInvalidValue;
  }
#undef MM_SPC
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

template <typename T, typename Tin, int LOGN, int V>
__global__ __attribute__((amdgpu_flat_work_group_size(1, OlsShape<LOGN, V>::NT),
                          amdgpu_waves_per_eu(OlsShape<LOGN, V>::WPE))) void k_ols(
    const Tin* __restrict__ yin, T* __restrict__ yout, const OlsChunk* __restrict__ chunks,
    const T* __restrict__ spec, const cx<T>* __restrict__ ptw, const cx<T>* __restrict__ tw2,
    int64_t n_t, int n_c, int m, const CgState* __restrict__ st) {
  using F = ShapeFFT<T, LOGN, V>;
  // Workgroups are dealt to the 8 XCDs round-robin in linear (x-fastest) order, so
  // XCD x takes workgroups x, x + 8, ...; give it a contiguous run of (RHS, chunk)
  // pairs instead, so that neighbouring chunks, whose windows overlap by 2 n_c
  // samples, read the shared samples through the same L2.
  const int64_t n_wg = (int64_t)gridDim.x * gridDim.y;
  const int64_t wl = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  const int64_t xq = n_wg >> 3, xr = n_wg & 7, xw = wl & 7;
  const int64_t job = xw * xq + (xw < xr ? xw : xr) + (wl >> 3);
  const int rhs = __builtin_amdgcn_readfirstlane((int)(job / gridDim.x));   // uniform: scalar row offsets
  if (st && !st[rhs].active) return;   // this RHS has stopped iterating
  using PI = typename PairU<Tin>::type;
  using PO = typename PairU<T>::type;
  __shared__ __align__(16) char lds[F::LDS_BYTES];
  constexpr int N = F::N, E = F::E, NT = F::NT;
  const int t = threadIdx.x;
  const OlsChunk ch = chunks[job - (int64_t)rhs * gridDim.x];
  const int64_t roff = (int64_t)rhs * n_t;
  const int64_t s0 = ch.out_start - n_c;
  const int64_t lo = ch.iv_lo, hi = ch.iv_hi;
  const Tin* __restrict__ src = yin + roff;

  cx<T> v[E];
  constexpr int L0 = F::first_log_fwd(), R0 = 1 << L0;
  // the window: whole inside the interval (pair accesses at any element boundary), cut
  // by an end of it (32-bit window offsets, samples [a, b) are data), or starting before
  // the TOD row (the first interval's first chunk)
  if (s0 >= lo && s0 + 2 * N <= hi) {
    const PI* __restrict__ src2 = reinterpret_cast<const PI*>(src + s0);
#pragma unroll
    for (int i = 0; i < E / R0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        // 32-bit offsets from the uniform window base: one VGPR per address
        const PI x = src2[(uint32_t)F::template in_index<L0>(t, i, r)];
        v[i * R0 + r] = {(T)x.x, (T)x.y};
      }
  } else if (s0 >= 0) {
    const Tin* __restrict__ base = src + s0;
    const int a = (int)(lo > s0 ? lo - s0 : 0);
    const int b = (int)(hi - s0 < 2 * N ? hi - s0 : 2 * N);
#pragma unroll
    for (int i = 0; i < E / R0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int k2 = 2 * F::template in_index<L0>(t, i, r);
        const T x = (k2 >= a && k2 < b) ? (T)base[(uint32_t)k2] : (T)0;
        const T y = (k2 + 1 >= a && k2 + 1 < b) ? (T)base[(uint32_t)(k2 + 1)] : (T)0;
        v[i * R0 + r] = {x, y};
      }
  } else {
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
  }

  F::forward(v, lds, ptw, t);

  // pair Z_k with Z_{N-k} (in registers, or through LDS) and apply the filter symbol.
  // For the pair (k, N-k): A = Z_k, B = conj Z_{N-k}, E = A + B, O = -i (A - B),
  // Y = (E + W O) F_k, Y' = (E - W O) F_{N-k}; the new Z_k is conj(s + i W^-1 d) and
  // the new Z_{N-k} is s - i W^-1 d, with s = Y + Y', d = Y - Y', W = e^{-2 pi i k/(2N)}.
  const T* __restrict__ S = spec + (int64_t)ch.filter * (N + 1);
  auto pair_terms = [&](int k, cx<T> A, cx<T> partner, cx<T>& sum, cx<T>& Wd) {
    const cx<T> B = cconj(partner);
    const cx<T> Ev = cadd(A, B);
    const cx<T> D = csub(A, B);
    const cx<T> O = {D.im, -D.re};            // -i (A - B)
    const cx<T> W = tw2[k];
    const cx<T> WO = cmul(W, O);
    const T sa = S[k], sb = S[N - k];
    const cx<T> Y = cscale(cadd(Ev, WO), sa);
    const cx<T> Yp = cscale(csub(Ev, WO), sb);
    sum = cadd(Y, Yp);
    Wd = cmul(cconj(W), csub(Y, Yp));          // W^{-k} (Y - Y')
  };
  if constexpr (F::PAIRED) {
    with_partner_paired<F>(v, t, [&](int k, cx<T>& zk, cx<T>& znk) {
      cx<T> sum, Wd;
      pair_terms(k, zk, znk, sum, Wd);
      zk = {sum.re - Wd.im, -(sum.im + Wd.re)};   // conj(sum + i Wd)
      znk = {sum.re + Wd.im, sum.im - Wd.re};     // sum - i Wd
    });
  } else {
    with_partner<F>(v, lds, t, [&](int k, cx<T> A, cx<T> partner) -> cx<T> {
      cx<T> sum, Wd;
      pair_terms(k, A, partner, sum, Wd);
      return {sum.re - Wd.im, -(sum.im + Wd.re)};
    });
  }

  F::forward_rev(v, lds, ptw, t);

  constexpr int LZ = F::last_log_rev(), RZ = 1 << LZ;
  // outputs 2j, 2j + 1 go to out_start + o, o = 2j - n_c, for o in [0, len): 32-bit offsets
  T* __restrict__ dst = yout + roff + ch.out_start;
  const int len = (int)(hi - ch.out_start < m ? hi - ch.out_start : m);   // outputs of this chunk
  if ((n_c & 1) == 0 && len == m) {   // whole pairs, all inside
    PO* __restrict__ dst2 = reinterpret_cast<PO*>(dst);
#pragma unroll
    for (int i = 0; i < E / RZ; ++i)
#pragma unroll
      for (int r = 0; r < RZ; ++r) {
        const int o = 2 * (t + i * NT + r * (N >> LZ)) - n_c;
        const cx<T> z = v[i * RZ + r];
        if (o >= 0 && o < m) dst2[(uint32_t)(o >> 1)] = PO{z.re, -z.im};
      }
  } else {
#pragma unroll
    for (int i = 0; i < E / RZ; ++i)
#pragma unroll
      for (int r = 0; r < RZ; ++r) {
        const int o = 2 * (t + i * NT + r * (N >> LZ)) - n_c;
        const cx<T> z = v[i * RZ + r];
        if (o >= 0 && o < len) dst[(uint32_t)o] = z.re;
        if (o + 1 >= 0 && o + 1 < len) dst[(uint32_t)(o + 1)] = -z.im;
      }
  }
}

template <typename T, typename Tin, int LOGN, int V = 0>
static hipError_t ols_launch(const void* y_in, void* y_out, const OlsChunk* chunks, int n_chunks,
                             const void* spec, const void* ptw, const void* tw2, int64_t n_t, int n_c,
                             int m, int n_rhs, hipStream_t s, const CgState* st) {
  hipLaunchKernelGGL((k_ols<T, Tin, LOGN, V>), dim3((unsigned)n_chunks, (unsigned)n_rhs),
                     dim3(OlsShape<LOGN, V>::NT), 0, s, (const Tin*)y_in, (T*)y_out, chunks,
                     (const T*)spec, (const cx<T>*)ptw, (const cx<T>*)tw2, n_t, n_c, m, st);
  return hipGetLastError();
}

template <typename T, typename Tin>
static hipError_t ols_dispatch(int logn, int variant, const void* y_in, void* y_out, const OlsChunk* chunks,
                               int n_chunks, const void* spec, const void* ptw, const void* tw2,
                               int64_t n_t, int n_c, int m, int n_rhs, hipStream_t s, const CgState* st) {
  if (!ols_variant_exists(logn, sizeof(T) == 8, variant)) return hipErrorInvalidValue;
  if (variant == 5) return ols_launch<T, Tin, 14, 5>(y_in, y_out, chunks, n_chunks, spec, ptw, tw2, n_t, n_c, m, n_rhs, s, st);
  if (variant == 7) return ols_launch<T, Tin, 14, 7>(y_in, y_out, chunks, n_chunks, spec, ptw, tw2, n_t, n_c, m, n_rhs, s, st);
  if (variant == 2 && logn == 14) return ols_launch<T, Tin, 14, 2>(y_in, y_out, chunks, n_chunks, spec, ptw, tw2, n_t, n_c, m, n_rhs, s, st);
#define MM_OLS_ARGS y_in, y_out, chunks, n_chunks, spec, ptw, tw2, n_t, n_c, m, n_rhs, s, st
  if constexpr (sizeof(T) == 4) {
    if (variant == 1)
      return logn == 13 ? ols_launch<T, Tin, 13, 1>(MM_OLS_ARGS)
                        : (logn == 14 ? ols_launch<T, Tin, 14, 1>(MM_OLS_ARGS) : ols_launch<T, Tin, 15, 1>(MM_OLS_ARGS));
    if (variant == 2) return logn == 14 ? ols_launch<T, Tin, 14, 2>(MM_OLS_ARGS) : ols_launch<T, Tin, 15, 2>(MM_OLS_ARGS);
    if (variant == 3) return ols_launch<T, Tin, 14, 3>(MM_OLS_ARGS);
    if (variant == 4) return ols_launch<T, Tin, 14, 4>(MM_OLS_ARGS);
    if (variant == 6) return ols_launch<T, Tin, 14, 6>(MM_OLS_ARGS);
    if (variant == 8) return ols_launch<T, Tin, 14, 8>(MM_OLS_ARGS);
    if (logn == 15) return ols_launch<T, Tin, 15>(MM_OLS_ARGS);
  }
#define MM_OLS_CASE(L) case L: return ols_launch<T, Tin, L>(MM_OLS_ARGS);
  switch (logn) {
    MM_OLS_CASE(6) MM_OLS_CASE(7) MM_OLS_CASE(8) MM_OLS_CASE(9) MM_OLS_CASE(10)
    MM_OLS_CASE(11) MM_OLS_CASE(12) MM_OLS_CASE(13) MM_OLS_CASE(14)
    default: break;
  }
#undef MM_OLS_CASE
#undef MM_OLS_ARGS
  return hipErrorInvalidValue;
}

hipError_t launch_ols(bool fp64, bool in_f64, int logn, const void* y_in, void* y_out,
                      const OlsChunk* chunks, int n_chunks, const void* spec, const void* ptw,
                      const void* tw2, int64_t n_t, int n_c, int m, int n_rhs, hipStream_t s, int variant,
                      const CgState* st) {
  if (n_chunks == 0 || n_rhs == 0) return hipSuccess;
  if (variant == 9) {
    if (fp64 || !ols_wave_exists(logn, fp64)) return hipErrorInvalidValue;
    return launch_ols_wave(logn, in_f64, y_in, y_out, chunks, n_chunks, spec, ptw, n_t, n_c, m, n_rhs, s, st);
  }
  if (fp64) {
    return in_f64 ? ols_dispatch<double, double>(logn, variant, y_in, y_out, chunks, n_chunks, spec, ptw, tw2,
                                                 n_t, n_c, m, n_rhs, s, st)
                  : ols_dispatch<double, float>(logn, variant, y_in, y_out, chunks, n_chunks, spec, ptw, tw2,
                                                n_t, n_c, m, n_rhs, s, st);
  }
  return in_f64 ? ols_dispatch<float, double>(logn, variant, y_in, y_out, chunks, n_chunks, spec, ptw, tw2, n_t,
                                              n_c, m, n_rhs, s, st)
                : ols_dispatch<float, float>(logn, variant, y_in, y_out, chunks, n_chunks, spec, ptw, tw2, n_t,
                                             n_c, m, n_rhs, s, st);
}

}  // namespace mm
