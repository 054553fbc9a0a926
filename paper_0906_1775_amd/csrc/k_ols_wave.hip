// Overlap-save N^-1 with a four-step 2^14-point transform whose inner stages stay
// inside one wavefront (float32, n_f = 2^15; the paper's transform is the chunked
// circulant embedding of its Weighting section).
//
// The 2^14 packed complex points z_n (n = g + 1024 n_o, thread g of 1024 holds
// n_o = 0..15) are transformed as
//   Z[k_o + 16 k_in] = sum_g W_1024^(g k_in) [ W_N^(g k_o) sum_n_o z[g + 1024 n_o] W_16^(n_o k_o) ]:
// 16-point DFTs in registers, one workgroup exchange that gives wavefront w the
// row k_o = w, then a 1024-point DFT of that row inside the wavefront (lane l and
// register j hold index l + 64 j): 16-point DFTs over j, a twiddle, an exchange
// through the wavefront's own LDS row, 4-point DFTs across lane groups, a twiddle,
// a second private exchange and 16-point DFTs.  Its output sits at lane mu,
// register c2 for index mu + 64 c2, which is the input layout of the same stage,
// so the inverse (a forward transform of the conjugate, read with the decomposition
// the other way round: 1024-point stage first, twiddle W_N^(n_a k_o), workgroup
// exchange, 16-point DFTs) reuses it.  Only three exchanges span the workgroup
// (the outer one of each transform and the real-to-complex pairing); the private
// ones need no barrier, so the wavefronts of a SIMD drift apart and one's exchanges
// overlap another's arithmetic.
//
// Pairing: Z_k (wavefront w, k_in) meets Z_(N-k) at wavefront 16 - w, 1023 - k_in
// (w = 0: wavefront 0, (1024 - k_in) mod 1024) through the LDS rows; the side with
// k_in < 512 forms both new points and writes its partner's back.  The symbol and the packing twiddle are read in the same row
// order (tables built by launch_wave_tables / launch_wave_symbols).
#include <algorithm>
#include <type_traits>

#include "fft.hpp"
#include "mm_internal.h"

namespace mm {

namespace {

constexpr int kWN = 1 << 14;      // complex points
constexpr int kWRow = 1088;       // LDS row stride (1024 + 64 padding for the second private exchange)
// table offsets (complex entries): twA[k * 1024 + g] = W_N^(g k), twB[k * 64 + l] = W_1024^(l k),
// twC[c * 16 + m] = W_64^(m c), twD[w * 1024 + n] = W_N^(w n), tw2[w * 1024 + k_in] = W_2N^(w + 16 k_in)
constexpr int kTA = 0, kTB = kWN, kTC = kTB + 1024, kTD = kTC + 64, kT2 = kTD + kWN, kTTotal = kT2 + kWN;

// l, opaque to the optimiser: table reads indexed by the result cannot be hoisted to the
// kernel's start (where they would stay live across the whole transform and spill)
// (the result is masked back to a lane index so that the compiler still knows its range
// and forms 32-bit offsets from the uniform table bases)
__device__ __forceinline__ int opaque(int l) {
  asm volatile("" : "+v"(l));
  return l & 63;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 16-point DFT in registers, natural order in and out, as 4 x 4:
// X[k1 + 4 k2] = sum_n2 W_4^(n2 k2) [ W_16^(n2 k1) sum_n1 x[n2 + 4 n1] W_4^(n1 k1) ]
// (8 4-point DFTs and 9 twiddles, one of them -i: 160 VALU operations against 168 for
// four radix-2 stages)
template <typename T>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  const cx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
  const cx<T> mt3 = {t3.im, -t3.re};   // -i t3
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, mt3);
  a3 = csub(t1, mt3);
}

template <typename T>
__device__ __forceinline__ void dft16(cx<T>* v) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);   // v[n2 + 4 k1]
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) v[n2 + 4 * k1] = twiddle_const(v[n2 + 4 * k1], n2 * k1, 16);
  cx<T> y[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<T> a0 = v[4 * k1], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
    dft4(a0, a1, a2, a3);
    y[k1] = a0;
    y[k1 + 4] = a1;
    y[k1 + 8] = a2;
    y[k1 + 12] = a3;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = y[k];
}

// 1024-point DFT of a wavefront's row: lane l, register j hold a[l + 64 j] on entry;
// lane mu, register c2 hold A[mu + 64 c2] on exit.  row: this wavefront's LDS row.
template <typename T>
__device__ __forceinline__ void inner_dft(cx<T>* v, cx<T>* row, const cx<T>* __restrict__ tab, int l) {
  // a[l + 64 j]: 16-point DFTs over j (output k1), twiddle W_1024^(l k1)
  l = opaque(l);
  dft16<T>(v);
#pragma unroll
  for (int k = 1; k < 16; ++k) v[k] = cmul(v[k], tab[(uint32_t)(kTB + k * 64 + l)]);
  // private exchange: value (k1, l) to k1 * 64 + l; lane (m, h) = (l & 15, l >> 4) takes
  // k1 = 4h + e and l' = m + 16 lh
  wave_sync();
#pragma unroll
  for (int k = 0; k < 16; ++k) row[k * 64 + l] = v[k];
  wave_sync();
  const int m = l & 15, h = l >> 4;
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int lh = 0; lh < 4; ++lh) v[e * 4 + lh] = row[(4 * h + e) * 64 + m + 16 * lh];
  // 4-point DFTs over lh (output c1), twiddle W_64^(m c1)
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    dft4(v[e * 4], v[e * 4 + 1], v[e * 4 + 2], v[e * 4 + 3]);
#pragma unroll
    for (int c = 1; c < 4; ++c) v[e * 4 + c] = cmul(v[e * 4 + c], tab[(uint32_t)(kTC + c * 16 + m)]);
  }
  // private exchange: value (k1, c1, m) to (c1 * 16 + k1) * 17 + m; lane mu = c1 * 16 + k1 takes m = 0..15
  wave_sync();
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int c = 0; c < 4; ++c) row[(c * 16 + 4 * h + e) * 17 + m] = v[e * 4 + c];
  wave_sync();
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = row[l * 17 + q];
  // 16-point DFTs over m (output c2): index k1 + 16 (c1 + 4 c2) = mu + 64 c2
  dft16<T>(v);
}

// The transpose of inner_dft's factorization, stage by stage in reverse order: lane mu =
// k1 + 16 c1, register c2 hold a[mu + 64 c2] on entry (inner_dft's output layout); lane l,
// register j hold A[l + 64 j] on exit.  The inverse transform runs this form, so that in
// floating point it is the transpose of the forward one and the float32 operator stays as
// symmetric as the exact one (the same DFT, with the rounding of the forward mirrored).
template <typename T>
__device__ __forceinline__ void inner_dft_t(cx<T>* v, cx<T>* row, const cx<T>* __restrict__ tab, int l) {
  l = opaque(l);
  // 16-point DFTs over c2 (output m), twiddle W_64^(m c1), c1 = mu >> 4
  dft16<T>(v);
  const int c1 = l >> 4;
#pragma unroll
  for (int q = 1; q < 16; ++q) v[q] = cmul(v[q], tab[(uint32_t)(kTC + c1 * 16 + q)]);
  // private exchange: value (k1, c1, m) at (c1 * 16 + k1) * 17 + m; lane (m, h) takes k1 = 4h + e, c1 = 0..3
  wave_sync();
#pragma unroll
  for (int q = 0; q < 16; ++q) row[l * 17 + q] = v[q];
  wave_sync();
  const int m = l & 15, h = l >> 4;
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int c = 0; c < 4; ++c) v[e * 4 + c] = row[(c * 16 + 4 * h + e) * 17 + m];
  // 4-point DFTs over c1 (output lh), twiddle W_1024^(l' k1), l' = m + 16 lh, k1 = 4h + e
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    dft4(v[e * 4], v[e * 4 + 1], v[e * 4 + 2], v[e * 4 + 3]);
#pragma unroll
    for (int lh = 0; lh < 4; ++lh)   // (k1 = 0 or l' = 0: the table holds exactly 1)
      v[e * 4 + lh] = cmul(v[e * 4 + lh], tab[(uint32_t)(kTB + (4 * h + e) * 64 + m + 16 * lh)]);
  }
  // private exchange: value (k1, l') at k1 * 64 + l'; lane l takes k1 = 0..15
  wave_sync();
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int lh = 0; lh < 4; ++lh) row[(4 * h + e) * 64 + m + 16 * lh] = v[e * 4 + lh];
  wave_sync();
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = row[k * 64 + l];
  // 16-point DFTs over k1 (output j)
  dft16<T>(v);
}

}  // namespace

bool ols_wave_exists(int logn, bool fp64) { return logn == 14 && !fp64; }
int ols_wave_table_count() { return kTTotal; }

// The packed window of one (chunk, RHS) job: thread g gets z[g + 1024 n_o] = u[2n] + i u[2n + 1]
template <typename Tin>
__device__ __forceinline__ void wave_load(cx<float>* v, const Tin* __restrict__ yin, const OlsChunk& ch, int rhs,
                                          int64_t n_t, int n_c, int g) {
  using T = float;
  using PI = typename std::conditional<sizeof(Tin) == 4, float2, double2>::type;
  const Tin* __restrict__ src = yin + (int64_t)rhs * n_t;
  const int64_t s0 = ch.out_start - n_c;
  const int64_t lo = ch.iv_lo, hi = ch.iv_hi;
  const bool in_inside = s0 >= lo && s0 + 2 * kWN <= hi &&
                         ((reinterpret_cast<uintptr_t>(src + s0) & (sizeof(PI) - 1)) == 0);
  if (in_inside) {
    const PI* __restrict__ src2 = reinterpret_cast<const PI*>(src + s0);
#pragma unroll
    for (int no = 0; no < 16; ++no) {
      const PI x = src2[(uint32_t)(g + 1024 * no)];
      v[no] = {(T)x.x, (T)x.y};
    }
  } else {
#pragma unroll
    for (int no = 0; no < 16; ++no) {
      const int64_t j = s0 + 2 * (int64_t)(g + 1024 * no);
      const T a = (j >= lo && j < hi) ? (T)src[j] : (T)0;
      const T b = (j + 1 >= lo && j + 1 < hi) ? (T)src[j + 1] : (T)0;
      v[no] = {a, b};
    }
  }
}

// N^-1 of one job whose window is in v (wave_load); writes the job's valid outputs.
__device__ __forceinline__ void wave_filter(cx<float>* v, cx<float>* lds, const OlsChunk ch, int rhs,
                                            float* __restrict__ yout, const float* __restrict__ spec_w,
                                            const cx<float>* __restrict__ tab, int64_t n_t, int n_c, int m,
                                            int g_in) {
  using T = float;
  constexpr int N = kWN;
  const int g = g_in, l = g_in & 63;
  const int w = __builtin_amdgcn_readfirstlane(g_in >> 6);   // wavefront index, uniform
  cx<T>* row = lds + w * kWRow;
  const int64_t s0 = ch.out_start - n_c;
  const int64_t hi = ch.iv_hi;
  // forward, outer stage: 16-point DFTs over n_o (output k_o), twiddle W_N^(g k_o)
  dft16<T>(v);
#pragma unroll
  for (int k = 1; k < 16; ++k) v[k] = cmul(v[k], tab[(uint32_t)(kTA + k * 1024 + g)]);
  // workgroup exchange: wavefront w takes row k_o = w, lane l the g = l + 64 j
#pragma unroll
  for (int k = 0; k < 16; ++k) lds[k * kWRow + g] = v[k];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = row[l + 64 * j];
  // forward, inner stage: lane mu, register c2 hold Z[w + 16 (mu + 64 c2)]
  inner_dft<T>(v, row, tab, l);

  // pairing with Z_(N-k) and the filter symbol (as k_ols: A = Z_k, B = conj Z_(N-k),
  // E = A + B, O = -i (A - B), Y = (E + W O) F_k, Y' = (E - W O) F_(N-k), s = Y + Y',
  // d = W^-1 (Y - Y'); the new Z_k is conj(s + i d), the new Z_(N-k) is s - i d).
  // Each wavefront forms both members of the pairs whose k_in < 512 (registers 0..7)
  // and writes the partner's member into the partner's row; it then reads its own
  // members with k_in >= 512 from its row.
  wave_sync();
#pragma unroll
  for (int c = 0; c < 16; ++c) row[l + 64 * c] = v[c];
  __syncthreads();
  const int wp = (16 - w) & 15;                 // partner wavefront
  cx<T>* prow = lds + wp * kWRow;
  const float* __restrict__ S = spec_w + (int64_t)ch.filter * (N + 1);
  const int lp = opaque(l);
  auto pair = [&](int kin, int kp, cx<T> A, cx<T> Bp, T sb, cx<T>& zk, cx<T>& znk) {
    const cx<T> B = cconj(Bp);
    const cx<T> Ev = cadd(A, B);
    const cx<T> D = csub(A, B);
    const cx<T> O = {D.im, -D.re};
    const cx<T> W = tab[(uint32_t)(kT2 + w * 1024 + kin)];
    const cx<T> WO = cmul(W, O);
    const T sa = S[(uint32_t)(w * 1024 + kin)];
    // (Y and Y' are formed with each symbol value on its own: combining sa +- sb first
    // would round a small F_k, where the 1/f filter suppresses, against a large F_(N-k))
    const cx<T> Y = cscale(cadd(Ev, WO), sa);
    const cx<T> Yp = cscale(csub(Ev, WO), sb);
    const cx<T> sm = cadd(Y, Yp);
    const cx<T> Wd = cmul(cconj(W), csub(Y, Yp));
    zk = {sm.re - Wd.im, -(sm.im + Wd.re)};
    znk = {sm.re + Wd.im, sm.im - Wd.re};
  };
  cx<T> other[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    // (four pairs at a time: the scheduler would otherwise hoist every table and
    // partner load and spill)
    if (c % 4 == 0) __builtin_amdgcn_sched_barrier(0);
    const int kin = lp + 64 * c;
    const int kp = w == 0 ? ((1024 - kin) & 1023) : 1023 - kin;   // partner's k_in
    const T sb = (w == 0 && kin == 0) ? S[N] : S[(uint32_t)(wp * 1024 + kp)];   // F_(N-k); k = 0 pairs with F_N
    pair(kin, kp, v[c], prow[kp], sb, v[c], other[c]);
  }
  // k = N/2 (wavefront 0, k_in = 512) is its own partner: lane 0 of wavefront 0
  cx<T> mid = v[8];
  if (w == 0 && lp == 0) {
    cx<T> unused;
    pair(512, 512, v[8], v[8], S[512], mid, unused);
  }
  wave_sync();   // this wavefront's partner-row reads precede its writes there
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int kin = lp + 64 * c;
    const int kp = w == 0 ? ((1024 - kin) & 1023) : 1023 - kin;
    if (!(w == 0 && kin == 0)) prow[kp] = other[c];   // k = 0 is its own partner
  }
  if (w == 0 && lp == 0) row[512] = mid;
  __syncthreads();
#pragma unroll
  for (int c = 8; c < 16; ++c) v[c] = row[l + 64 * c];

  // inverse: forward transform of the conjugated spectrum, the transpose of the forward
  // one: inner stage first (input index k_in = mu + 64 c2, output n_a = l + 64 j), then
  // twiddle W_N^(n_a k_o) with k_o = w
  inner_dft_t<T>(v, row, tab, l);
  const int ld = opaque(l);
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    if (c % 8 == 0) __builtin_amdgcn_sched_barrier(0);
    v[c] = cmul(v[c], tab[(uint32_t)(kTD + w * 1024 + ld + 64 * c)]);
  }
  wave_sync();
#pragma unroll
  for (int c = 0; c < 16; ++c) row[l + 64 * c] = v[c];
  __syncthreads();
  // thread g = n_a takes k_o = 0..15; 16-point DFTs over k_o give X[g + 1024 n_b]
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = lds[k * kWRow + g];
  dft16<T>(v);

  // outputs 2n, 2n + 1 of n = g + 1024 n_b: the conjugate (re, -im)
  T* __restrict__ dst = yout + (int64_t)rhs * n_t;
  const bool out_inside = ((n_c & 1) == 0) && s0 + n_c + m <= hi &&
                          ((reinterpret_cast<uintptr_t>(dst + s0) & (sizeof(float2) - 1)) == 0);
  if (out_inside) {
    float2* __restrict__ dst2 = reinterpret_cast<float2*>(dst + s0);
    const int j0 = n_c >> 1, j1 = (n_c + m) >> 1;
#pragma unroll
    for (int nb = 0; nb < 16; ++nb) {
      const int j = g + 1024 * nb;
      if (j >= j0 && j < j1) dst2[(uint32_t)j] = float2{v[nb].re, -v[nb].im};
    }
  } else {
#pragma unroll
    for (int nb = 0; nb < 16; ++nb) {
      const int pos = 2 * (g + 1024 * nb);
      if (pos >= n_c && pos < n_c + m && s0 + pos < hi) dst[s0 + pos] = v[nb].re;
      if (pos + 1 >= n_c && pos + 1 < n_c + m && s0 + pos + 1 < hi) dst[s0 + pos + 1] = -v[nb].im;
    }
  }
}


// One workgroup per (chunk, RHS), as k_ols (same XCD-aware order, same outputs).
template <typename Tin>
__global__ __launch_bounds__(1024) void k_ols_wave(const Tin* __restrict__ yin, float* __restrict__ yout,
                                                   const OlsChunk* __restrict__ chunks,
                                                   const float* __restrict__ spec_w,
                                                   const cx<float>* __restrict__ tab, int64_t n_t, int n_c, int m,
                                                   const CgState* __restrict__ st) {
  const int64_t n_wg = (int64_t)gridDim.x * gridDim.y;
  const int64_t wl = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  const int64_t xq = n_wg >> 3, xr = n_wg & 7, xw = wl & 7;
  const int64_t job = xw * xq + (xw < xr ? xw : xr) + (wl >> 3);
  const int rhs = (int)(job / gridDim.x);
  if (st && !st[rhs].active) return;   // this RHS has stopped iterating
  __shared__ __align__(16) cx<float> lds[16 * kWRow];
  const OlsChunk ch = chunks[job - (int64_t)rhs * gridDim.x];
  cx<float> v[16];
  wave_load<Tin>(v, yin, ch, rhs, n_t, n_c, threadIdx.x);
  wave_filter(v, lds, ch, rhs, yout, spec_w, tab, n_t, n_c, m, threadIdx.x);
}

// Twiddle tables of k_ols_wave, float32 from float64 angles
__global__ void k_wave_tables(cx<float>* __restrict__ tab) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kTTotal) return;
  double num, den;   // angle = -2 pi num / den
  if (e < kTB) { const int k = e / 1024, g = e % 1024; num = (double)g * k; den = kWN; }
  else if (e < kTC) { const int k = (e - kTB) / 64, l = (e - kTB) % 64; num = (double)l * k; den = 1024; }
  else if (e < kTD) { const int c = (e - kTC) / 16, m = (e - kTC) % 16; num = (double)m * c; den = 64; }
  else if (e < kT2) { const int w = (e - kTD) / 1024, n = (e - kTD) % 1024; num = (double)w * n; den = kWN; }
  else { const int w = (e - kT2) / 1024, kin = (e - kT2) % 1024; num = (double)(w + 16 * kin); den = 2.0 * kWN; }
  const double frac = num / den;
  double sn, cs;
  sincospi(2.0 * (frac - floor(frac)), &sn, &cs);
  tab[e] = {(float)cs, (float)(-sn)};
}

// spec_w[f][w * 1024 + k_in] = spec[f][w + 16 k_in], spec_w[f][N] = spec[f][N]
__global__ void k_wave_symbols(const float* __restrict__ spec, float* __restrict__ spec_w) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > kWN) return;
  const float* __restrict__ src = spec + (int64_t)blockIdx.y * (kWN + 1);
  float* __restrict__ dst = spec_w + (int64_t)blockIdx.y * (kWN + 1);
  dst[e] = e == kWN ? src[kWN] : src[(e >> 10) + 16 * (e & 1023)];
}

hipError_t launch_wave_tables(void* tab, hipStream_t s) {
  hipLaunchKernelGGL(k_wave_tables, dim3((kTTotal + 255) / 256), dim3(256), 0, s, (cx<float>*)tab);
  return hipGetLastError();
}

hipError_t launch_wave_symbols(const void* spec, void* spec_w, int n_filters, hipStream_t s) {
  if (n_filters <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_wave_symbols, dim3((kWN + 1 + 255) / 256, (unsigned)n_filters), dim3(256), 0, s,
                     (const float*)spec, (float*)spec_w);
  return hipGetLastError();
}

hipError_t launch_ols_wave(bool in_f64, const void* y_in, void* y_out, const OlsChunk* chunks, int n_chunks,
                           const void* spec_w, const void* tab, int64_t n_t, int n_c, int m, int n_rhs,
                           hipStream_t s, const CgState* st) {
  if (n_chunks == 0 || n_rhs == 0) return hipSuccess;
  const dim3 grid((unsigned)n_chunks, (unsigned)n_rhs);
  if (in_f64)
    hipLaunchKernelGGL(k_ols_wave<double>, grid, dim3(1024), 0, s, (const double*)y_in, (float*)y_out, chunks,
                       (const float*)spec_w, (const cx<float>*)tab, n_t, n_c, m, st);
  else
    hipLaunchKernelGGL(k_ols_wave<float>, grid, dim3(1024), 0, s, (const float*)y_in, (float*)y_out, chunks,
                       (const float*)spec_w, (const cx<float>*)tab, n_t, n_c, m, st);
  return hipGetLastError();
}

}  // namespace mm
