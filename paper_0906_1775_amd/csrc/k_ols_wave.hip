// Overlap-save N^-1 with four-step transforms of 2^14 and 2^15 points whose inner
// stages stay inside one wavefront (float32, n_f = 2^15 and 2^16; the paper's transform
// is the chunked circulant embedding of its Weighting section).
//
// The N = 1024 NO packed complex points z_n (n = g + 1024 n_o, thread g of 1024 holds
// n_o = 0..NO-1; NO = 16 or 32) are transformed as
//   Z[k_o + NO k_in] = sum_g W_1024^(g k_in) [ W_N^(g k_o) sum_n_o z[g + 1024 n_o] W_NO^(n_o k_o) ]:
// NO-point DFTs in registers, a workgroup exchange that gives wavefront w the row k_o = w
// (and, for NO = 32, the row w + 16: the exchange then runs in two halves), then a
// 1024-point DFT of each row inside the wavefront (lane l and register j hold index
// l + 64 j): 16-point DFTs over j, a twiddle, an exchange through the wavefront's own LDS
// row, 4-point DFTs across lane groups, a twiddle, a second private exchange and 16-point
// DFTs.  Its output sits at lane mu, register c2 for index mu + 64 c2, which is the input
// layout of the same stage, so the inverse (a forward transform of the conjugate, read
// with the decomposition the other way round: 1024-point stage first, twiddle
// W_N^(n_a k_o), workgroup exchange, NO-point DFTs) reuses it.  Only the outer exchanges
// of each transform and the real-to-complex pairing span the workgroup; the private ones
// need no barrier, so the wavefronts of a SIMD drift apart and one's exchanges overlap
// another's arithmetic.
//
// Pairing: Z_k (row k_o, k_in) meets Z_(N-k) at row NO - k_o, 1023 - k_in (row 0: row 0,
// (1024 - k_in) mod 1024) through the LDS rows.  For NO = 16 the side with k_in < 512
// forms both new points and writes its partner's back; for NO = 32 wavefront w >= 1 forms
// every pair of its row w with row 32 - w (wavefront 16 - w's second row, which waits in
// LDS), and wavefront 0 pairs rows 0 and 16 within themselves.  The symbol and the packing
// twiddle are read in the same row order (tables built by launch_wave_tables /
// launch_wave_symbols).
#include <algorithm>
#include <type_traits>

#include "fft.hpp"
#include "mm_internal.h"

namespace mm {

namespace {

constexpr int kWN = 1 << 14;      // complex points of the 16 x 1024 transform
constexpr int kWN32 = 1 << 15;    // complex points of the 32 x 1024 transform
constexpr int kWRow = 1088;       // LDS row stride (1024 + 64 padding for the second private exchange)
// table offsets (complex entries): twB[k * 64 + l] = W_1024^(l k), twC[c * 16 + m] = W_64^(m c),
// twA[k * 1024 + g] = W_N^(g k) (k < NO; the forward's outer twiddle and the inverse's),
// tw2[r * 1024 + k_in] = W_2N^(r + NO k_in) (r < NO)
constexpr int kTB = 0, kTC = 1024, kTA = 1088;
constexpr int wave_t2(int logn) { return kTA + (1 << logn); }
constexpr int wave_table_total(int logn) { return kTA + 2 * (1 << logn); }
constexpr int kT2 = wave_t2(14);

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

// 32-point DFT in registers, natural order in and out: radix-2 butterflies of n and
// n + 16 with W_32^n on the differences, then two 16-point DFTs:
// X[2 k + b] = sum_n W_16^(n k) [ W_32^(n b) (x[n] + (-1)^b x[n + 16]) ]
template <typename T>
__device__ __forceinline__ void dft32(cx<T>* v) {
  cx<T> e[16], o[16];
#pragma unroll
  for (int n = 0; n < 16; ++n) {
    e[n] = cadd(v[n], v[n + 16]);
    o[n] = twiddle_const(csub(v[n], v[n + 16]), n, 32);
  }
  dft16<T>(e);
  dft16<T>(o);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    v[2 * k] = e[k];
    v[2 * k + 1] = o[k];
  }
}

// dft32's factorization transposed (the same DFT): 16-point DFTs of the even and odd
// inputs, W_32^n on the odd ones, radix-2 butterflies X[n], X[n + 16]
template <typename T>
__device__ __forceinline__ void dft32_t(cx<T>* v) {
  cx<T> e[16], o[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    e[k] = v[2 * k];
    o[k] = v[2 * k + 1];
  }
  dft16<T>(e);
  dft16<T>(o);
#pragma unroll
  for (int n = 0; n < 16; ++n) {
    const cx<T> t = twiddle_const(o[n], n, 32);
    v[n] = cadd(e[n], t);
    v[n + 16] = csub(e[n], t);
  }
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


// The packed window of one (chunk, RHS) job: thread g gets z[g + 1024 n_o] = u[2n] + i u[2n + 1],
// n_o < NO, u[i] = TOD sample s0 + i inside the chunk's interval, else 0 (s0 = out_start - n_c).
// Offsets inside the window are 32-bit from its first sample.
template <typename Tin, int NO>
__device__ __forceinline__ void wave_load(cx<float>* v, const Tin* __restrict__ yin, const OlsChunk& ch, int rhs,
                                          int64_t n_t, int n_c, int g) {
  using T = float;
  using PU = typename PairU<Tin>::type;
  constexpr int W = 2048 * NO;   // window samples
  const Tin* __restrict__ src = yin + (int64_t)rhs * n_t;
  const int64_t s0 = ch.out_start - n_c;
  const int64_t lo = ch.iv_lo, hi = ch.iv_hi;
  if (s0 >= lo && s0 + W <= hi) {   // the whole window inside the interval
    const PU* __restrict__ b2 = reinterpret_cast<const PU*>(src + s0);
#pragma unroll
    for (int no = 0; no < NO; ++no) {
      const PU x = b2[(uint32_t)(g + 1024 * no)];
      v[no] = {(T)x.x, (T)x.y};
    }
  } else if (s0 >= 0) {   // a window cut by an end of the interval: samples [a, b) of it are data
    const Tin* __restrict__ base = src + s0;
    const int a = (int)(lo > s0 ? lo - s0 : 0);
    const int b = (int)(hi - s0 < W ? hi - s0 : W);
#pragma unroll
    for (int no = 0; no < NO; ++no) {
      const int i = 2 * (g + 1024 * no);
      const T x = (i >= a && i < b) ? (T)base[(uint32_t)i] : (T)0;
      const T y = (i + 1 >= a && i + 1 < b) ? (T)base[(uint32_t)(i + 1)] : (T)0;
      v[no] = {x, y};
    }
  } else {   // the window starts before the TOD row (the first interval's first chunk)
#pragma unroll
    for (int no = 0; no < NO; ++no) {
      const int64_t j = s0 + 2 * (int64_t)(g + 1024 * no);
      const T a = (j >= lo && j < hi) ? (T)src[j] : (T)0;
      const T b = (j + 1 >= lo && j + 1 < hi) ? (T)src[j + 1] : (T)0;
      v[no] = {a, b};
    }
  }
}

// Outputs 2n, 2n + 1 of n = g + 1024 n_b (n_b < NO) of one job: the conjugate (re, -im) of
// v[n_b]; window positions [n_c, n_c + m) are the chunk's outputs, out_start onwards, cut at
// the interval's end.  Offsets are 32-bit from out_start.
template <int NO>
__device__ __forceinline__ void wave_store(const cx<float>* v, float* __restrict__ yout, const OlsChunk& ch,
                                           int rhs, int64_t n_t, int n_c, int m, int g) {
  float* __restrict__ base = yout + (int64_t)rhs * n_t + ch.out_start;
  const int len = (int)(ch.iv_hi - ch.out_start < m ? ch.iv_hi - ch.out_start : m);   // outputs of this chunk
  if ((n_c & 1) == 0 && len == m) {   // whole pairs, all inside
    FloatPairU* __restrict__ b2 = reinterpret_cast<FloatPairU*>(base);
#pragma unroll
    for (int nb = 0; nb < NO; ++nb) {
      const int j = 2 * (g + 1024 * nb) - n_c;
      if (j >= 0 && j < m) b2[(uint32_t)(j >> 1)] = FloatPairU{v[nb].re, -v[nb].im};
    }
  } else {
#pragma unroll
    for (int nb = 0; nb < NO; ++nb) {
      const int j = 2 * (g + 1024 * nb) - n_c;
      if (j >= 0 && j < len) base[(uint32_t)j] = v[nb].re;
      if (j + 1 >= 0 && j + 1 < len) base[(uint32_t)(j + 1)] = -v[nb].im;
    }
  }
}

// One conjugate pair of the real-to-complex step with the filter symbol (as k_ols):
// A = Z_k, B = conj Z_(N-k), E = A + B, O = -i (A - B), Y = (E + W O) F_k,
// Y' = (E - W O) F_(N-k), s = Y + Y', d = W^-1 (Y - Y'); the new Z_k is conj(s + i d),
// the new Z_(N-k) is s - i d.  W = W_2N^k, sa = F_k / (4N), sb = F_(N-k) / (4N).
// (Y and Y' are formed with each symbol value on its own: combining sa +- sb first
// would round a small F_k, where the 1/f filter suppresses, against a large F_(N-k).)
__device__ __forceinline__ void wave_pair(cx<float> A, cx<float> Bp, cx<float> W, float sa, float sb,
                                          cx<float>& zk, cx<float>& znk) {
  using T = float;
  const cx<T> B = cconj(Bp);
  const cx<T> Ev = cadd(A, B);
  const cx<T> D = csub(A, B);
  const cx<T> O = {D.im, -D.re};
  const cx<T> WO = cmul(W, O);
  const cx<T> Y = cscale(cadd(Ev, WO), sa);
  const cx<T> Yp = cscale(csub(Ev, WO), sb);
  const cx<T> sm = cadd(Y, Yp);
  const cx<T> Wd = cmul(cconj(W), csub(Y, Yp));
  zk = {sm.re - Wd.im, -(sm.im + Wd.re)};
  znk = {sm.re + Wd.im, sm.im - Wd.re};
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

  // pairing with Z_(N-k) and the filter symbol (wave_pair).
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
    wave_pair(A, Bp, tab[(uint32_t)(kT2 + w * 1024 + kin)], S[(uint32_t)(w * 1024 + kin)], sb, zk, znk);
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
    v[c] = cmul(v[c], tab[(uint32_t)(kTA + w * 1024 + ld + 64 * c)]);
  }
  wave_sync();
#pragma unroll
  for (int c = 0; c < 16; ++c) row[l + 64 * c] = v[c];
  __syncthreads();
  // thread g = n_a takes k_o = 0..15; 16-point DFTs over k_o give X[g + 1024 n_b]
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = lds[k * kWRow + g];
  dft16<T>(v);

  wave_store<16>(v, yout, ch, rhs, n_t, n_c, m, g);
}


// N^-1 of one job of the 32 x 1024 transform whose window is in v[32] (wave_load); writes
// the job's valid outputs.  Wavefront w holds rows w (va) and w + 16 (vb) between the outer
// stages; lds has 17 rows (the 17th takes row 0 during the pairing).
__device__ __forceinline__ void wave_filter32(cx<float>* v, cx<float>* lds, const OlsChunk ch, int rhs,
                                              float* __restrict__ yout, const float* __restrict__ spec_w,
                                              const cx<float>* __restrict__ tab, int64_t n_t, int n_c, int m,
                                              int g_in) {
  using T = float;
  constexpr int N = kWN32;
  constexpr int T2 = wave_t2(15);
  const int g = g_in, l = g_in & 63;
  const int w = __builtin_amdgcn_readfirstlane(g_in >> 6);   // wavefront index, uniform
  cx<T>* row = lds + w * kWRow;
  // forward, outer stage: 32-point DFTs over n_o (output k_o), twiddle W_N^(g k_o)
  dft32<T>(v);
#pragma unroll
  for (int k = 1; k < 32; ++k) {
    if (k % 8 == 0) __builtin_amdgcn_sched_barrier(0);
    v[k] = cmul(v[k], tab[(uint32_t)(kTA + k * 1024 + g)]);
  }
  // workgroup exchange in two halves: wavefront w takes row k_o = w, then k_o = w + 16
  cx<T> va[16], vb[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) lds[k * kWRow + g] = v[k];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) va[j] = row[l + 64 * j];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 16; ++k) lds[k * kWRow + g] = v[16 + k];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) vb[j] = row[l + 64 * j];
  // forward, inner stages: lane mu, register c2 hold Z[r + 32 (mu + 64 c2)], r = w, w + 16
  inner_dft<T>(va, row, tab, l);
  inner_dft<T>(vb, row, tab, l);

  // pairing with Z_(N-k) and the filter symbol (wave_pair).  The second rows wait in the
  // LDS rows (wavefront 0 also puts its row 0 in the 17th); wavefront w >= 1 forms every pair
  // of its row w (k_in) with row 32 - w (k_in' = 1023 - k_in, in wavefront 16 - w's LDS row),
  // keeps its own members and writes the partner's back; wavefront 0 pairs row 16 (k_in <
  // 512 with 1023 - k_in) and row 0 (k_in <= 512 with (1024 - k_in) mod 1024) in place.
  // Every LDS entry of the phase is read and written by one lane only.
  const float* __restrict__ S = spec_w + (int64_t)ch.filter * (N + 1);
  cx<T>* row0 = lds + 16 * kWRow;
  wave_sync();
#pragma unroll
  for (int c = 0; c < 16; ++c) row[l + 64 * c] = vb[c];
  if (w == 0) {
#pragma unroll
    for (int c = 0; c < 16; ++c) row0[l + 64 * c] = va[c];
  }
  __syncthreads();
  const int lp = opaque(l);
  if (w != 0) {
    const int r = w, rp = 32 - w;
    cx<T>* prow = lds + (16 - w) * kWRow;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      // (four pairs at a time: the scheduler would otherwise hoist every table and
      // partner load and spill)
      if (c % 4 == 0) __builtin_amdgcn_sched_barrier(0);
      const int kin = lp + 64 * c, kp = 1023 - kin;
      cx<T> znk;
      wave_pair(va[c], prow[kp], tab[(uint32_t)(T2 + r * 1024 + kin)], S[(uint32_t)(r * 1024 + kin)],
                S[(uint32_t)(rp * 1024 + kp)], va[c], znk);
      prow[kp] = znk;
    }
  } else {
#pragma unroll
    for (int c = 0; c < 8; ++c) {   // row 16 with itself (in this wavefront's LDS row)
      if (c % 4 == 0) __builtin_amdgcn_sched_barrier(0);
      const int kin = lp + 64 * c, kp = 1023 - kin;
      cx<T> zk, znk;
      wave_pair(row[kin], row[kp], tab[(uint32_t)(T2 + 16 * 1024 + kin)], S[(uint32_t)(16 * 1024 + kin)],
                S[(uint32_t)(16 * 1024 + kp)], zk, znk);
      row[kin] = zk;
      row[kp] = znk;
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {   // row 0 with itself; k = 0 pairs with F_N
      if (c % 4 == 0) __builtin_amdgcn_sched_barrier(0);
      const int kin = lp + 64 * c, kp = (1024 - kin) & 1023;
      cx<T> zk, znk;
      wave_pair(row0[kin], row0[kp], tab[(uint32_t)(T2 + kin)], S[(uint32_t)kin],
                kin == 0 ? S[N] : S[(uint32_t)kp], zk, znk);
      row0[kin] = zk;
      if (kin != 0) row0[kp] = znk;
    }
    if (lp == 0) {   // k = N/2 (row 0, k_in = 512) is its own partner
      const cx<T> a = row0[512];
      cx<T> zk, unused;
      wave_pair(a, a, tab[(uint32_t)(T2 + 512)], S[512], S[512], zk, unused);
      row0[512] = zk;
    }
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int c = 0; c < 16; ++c) va[c] = row0[l + 64 * c];
  }
#pragma unroll
  for (int c = 0; c < 16; ++c) vb[c] = row[l + 64 * c];

  // inverse: forward transform of the conjugated spectrum, the transpose of the forward
  // one: inner stages first (input index k_in = mu + 64 c2, output n_a = l + 64 j), twiddle
  // W_N^(n_a k_o) with k_o = w, w + 16
  const int ld = opaque(l);
  inner_dft_t<T>(va, row, tab, l);
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    if (c % 8 == 0) __builtin_amdgcn_sched_barrier(0);
    va[c] = cmul(va[c], tab[(uint32_t)(kTA + w * 1024 + ld + 64 * c)]);
  }
  inner_dft_t<T>(vb, row, tab, l);
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    if (c % 8 == 0) __builtin_amdgcn_sched_barrier(0);
    vb[c] = cmul(vb[c], tab[(uint32_t)(kTA + (w + 16) * 1024 + ld + 64 * c)]);
  }
  // workgroup exchange in two halves: thread g = n_a takes k_o = 0..15, then 16..31
  wave_sync();
#pragma unroll
  for (int c = 0; c < 16; ++c) row[l + 64 * c] = va[c];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = lds[k * kWRow + g];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 16; ++c) row[l + 64 * c] = vb[c];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 16; ++k) v[16 + k] = lds[k * kWRow + g];
  // 32-point DFTs over k_o (the forward's outer factorization transposed) give X[g + 1024 n_b]
  dft32_t<T>(v);
  wave_store<32>(v, yout, ch, rhs, n_t, n_c, m, g);
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
  const int rhs = __builtin_amdgcn_readfirstlane((int)(job / gridDim.x));   // uniform: scalar row offsets
  if (st && !st[rhs].active) return;   // this RHS has stopped iterating
  __shared__ __align__(16) cx<float> lds[16 * kWRow];
  const OlsChunk ch = chunks[job - (int64_t)rhs * gridDim.x];
  cx<float> v[16];
  wave_load<Tin, 16>(v, yin, ch, rhs, n_t, n_c, threadIdx.x);
  wave_filter(v, lds, ch, rhs, yout, spec_w, tab, n_t, n_c, m, threadIdx.x);
}

// One workgroup per (chunk, RHS) of the 32 x 1024 transform, as k_ols_wave
template <typename Tin>
__global__ __launch_bounds__(1024) void k_ols_wave32(const Tin* __restrict__ yin, float* __restrict__ yout,
                                                     const OlsChunk* __restrict__ chunks,
                                                     const float* __restrict__ spec_w,
                                                     const cx<float>* __restrict__ tab, int64_t n_t, int n_c,
                                                     int m, const CgState* __restrict__ st) {
  const int64_t n_wg = (int64_t)gridDim.x * gridDim.y;
  const int64_t wl = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  const int64_t xq = n_wg >> 3, xr = n_wg & 7, xw = wl & 7;
  const int64_t job = xw * xq + (xw < xr ? xw : xr) + (wl >> 3);
  const int rhs = __builtin_amdgcn_readfirstlane((int)(job / gridDim.x));   // uniform: scalar row offsets
  if (st && !st[rhs].active) return;   // this RHS has stopped iterating
  __shared__ __align__(16) cx<float> lds[17 * kWRow];
  const OlsChunk ch = chunks[job - (int64_t)rhs * gridDim.x];
  cx<float> v[32];
  wave_load<Tin, 32>(v, yin, ch, rhs, n_t, n_c, threadIdx.x);
  wave_filter32(v, lds, ch, rhs, yout, spec_w, tab, n_t, n_c, m, threadIdx.x);
}

// Twiddle tables of the 2^LOGN-point transform, float32 from float64 angles
template <int LOGN>
__global__ void k_wave_tables(cx<float>* __restrict__ tab) {
  constexpr int N = 1 << LOGN, NO = N / 1024, T2 = wave_t2(LOGN);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= wave_table_total(LOGN)) return;
  double num, den;   // angle = -2 pi num / den
  if (e < kTC) { const int k = e / 64, l = e % 64; num = (double)l * k; den = 1024; }
  else if (e < kTA) { const int c = (e - kTC) / 16, m = (e - kTC) % 16; num = (double)m * c; den = 64; }
  else if (e < T2) { const int k = (e - kTA) / 1024, g = (e - kTA) % 1024; num = (double)g * k; den = N; }
  else { const int r = (e - T2) / 1024, kin = (e - T2) % 1024; num = (double)(r + NO * kin); den = 2.0 * N; }
  const double frac = num / den;
  double sn, cs;
  sincospi(2.0 * (frac - floor(frac)), &sn, &cs);
  tab[e] = {(float)cs, (float)(-sn)};
}

// spec_w[f][r * 1024 + k_in] = spec[f][r + NO k_in], spec_w[f][N] = spec[f][N]
template <int LOGN>
__global__ void k_wave_symbols(const float* __restrict__ spec, float* __restrict__ spec_w) {
  constexpr int N = 1 << LOGN, NO = N / 1024;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > N) return;
  const float* __restrict__ src = spec + (int64_t)blockIdx.y * (N + 1);
  float* __restrict__ dst = spec_w + (int64_t)blockIdx.y * (N + 1);
  dst[e] = e == N ? src[N] : src[(e >> 10) + NO * (e & 1023)];
}

}  // namespace

bool ols_wave_exists(int logn, bool fp64) { return (logn == 14 || logn == 15) && !fp64; }
int ols_wave_table_count(int logn) { return wave_table_total(logn); }

hipError_t launch_wave_tables(int logn, void* tab, hipStream_t s) {
  if (!ols_wave_exists(logn, false)) return hipErrorInvalidValue;
  const int n = wave_table_total(logn);
  if (logn == 14)
    hipLaunchKernelGGL(k_wave_tables<14>, dim3((n + 255) / 256), dim3(256), 0, s, (cx<float>*)tab);
  else
    hipLaunchKernelGGL(k_wave_tables<15>, dim3((n + 255) / 256), dim3(256), 0, s, (cx<float>*)tab);
  return hipGetLastError();
}

hipError_t launch_wave_symbols(int logn, const void* spec, void* spec_w, int n_filters, hipStream_t s) {
  if (!ols_wave_exists(logn, false)) return hipErrorInvalidValue;
  if (n_filters <= 0) return hipSuccess;
  const dim3 grid(((1 << logn) + 1 + 255) / 256, (unsigned)n_filters);
  if (logn == 14)
    hipLaunchKernelGGL(k_wave_symbols<14>, grid, dim3(256), 0, s, (const float*)spec, (float*)spec_w);
  else
    hipLaunchKernelGGL(k_wave_symbols<15>, grid, dim3(256), 0, s, (const float*)spec, (float*)spec_w);
  return hipGetLastError();
}

hipError_t launch_ols_wave(int logn, bool in_f64, const void* y_in, void* y_out, const OlsChunk* chunks,
                           int n_chunks, const void* spec_w, const void* tab, int64_t n_t, int n_c, int m,
                           int n_rhs, hipStream_t s, const CgState* st) {
  if (!ols_wave_exists(logn, false)) return hipErrorInvalidValue;
  if (n_chunks == 0 || n_rhs == 0) return hipSuccess;
  const dim3 grid((unsigned)n_chunks, (unsigned)n_rhs);
  const float* sw = (const float*)spec_w;
  const cx<float>* tw = (const cx<float>*)tab;
  if (logn == 14 && in_f64)
    hipLaunchKernelGGL(k_ols_wave<double>, grid, dim3(1024), 0, s, (const double*)y_in, (float*)y_out, chunks, sw,
                       tw, n_t, n_c, m, st);
  else if (logn == 14)
    hipLaunchKernelGGL(k_ols_wave<float>, grid, dim3(1024), 0, s, (const float*)y_in, (float*)y_out, chunks, sw,
                       tw, n_t, n_c, m, st);
  else if (in_f64)
    hipLaunchKernelGGL(k_ols_wave32<double>, grid, dim3(1024), 0, s, (const double*)y_in, (float*)y_out, chunks,
                       sw, tw, n_t, n_c, m, st);
  else
    hipLaunchKernelGGL(k_ols_wave32<float>, grid, dim3(1024), 0, s, (const float*)y_in, (float*)y_out, chunks,
                       sw, tw, n_t, n_c, m, st);
  return hipGetLastError();
}

}  // namespace mm
