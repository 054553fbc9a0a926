// Workgroup-resident complex FFT for gfx950 (device code).
//
// A workgroup of NT threads transforms N = 2^LOGN complex points.  Each
// thread keeps E = N / NT points in registers; the transform is a sequence of
// Stockham autosort passes (radix 2^LOGE, plus one shorter pass when LOGE
// does not divide LOGN).  A pass runs the radix-R butterflies of one thread
// entirely in registers; between passes the points are re-distributed
// through LDS (all at once when N complex points fit, else real parts then
// imaginary parts through an N-scalar buffer).  LDS indices are padded by one
// element per 128-byte row so the strided writes of the early passes spread
// over the banks.
//
// Pass with radix R and span Ns (product of the radices before it), for
// butterfly b in [0, N/R) and element r in [0, R):
//   input  index  b + r N/R,
//   twiddle       exp(-2 pi i (b mod Ns) r / (Ns R)),
//   output index  (b / Ns) Ns R + (b mod Ns) + r Ns.
// Thread t owns butterflies b = t + i NT.  After the last pass the output of
// (b, r) is point b + r N/R_last, i.e. the natural order, strided.
//
// Paired layout (PAIRED, for shapes with an even number NB of butterflies per
// thread in the last forward pass): there thread t > 0 owns butterflies
// t + i NT (i even) and (NB - i + 1) NT - t (i odd), and thread 0 owns i NT,
// instead of t + i NT.  Butterflies b and N/R - b hold the points k and N - k,
// so after the forward transform every thread has both members of its
// conjugate pairs (Z_k, Z_{N-k}) in registers.  The first pass of the
// radix-reversed sequence shares that layout.
//
// Twiddles come from per-pass tables built once in float64 and rounded to T:
// pass p with radix R and span Ns owns Ns rows of R entries,
// row j = exp(-2 pi i j r / (Ns R)), r < R, so a thread reads its R-1 factors
// as one contiguous row.  The forward and the radix-reversed sequences have
// their own tables (tw_offset).  A second table tw2[k] = exp(-2 pi i k/(2N)),
// k < N, serves the real-to-complex packing of the overlap-save filter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mm {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
// Pairs of TOD elements at any element boundary (windows of intervals that start at an
// odd sample): 4- and 8-byte aligned, where float2 / double2 need 8 and 16 (the loads and
// stores are still single 8- and 16-byte accesses)
struct alignas(4) FloatPairU { float x, y; };
struct alignas(8) DoublePairU { double x, y; };
template <typename T> struct PairU;
template <> struct PairU<float> { using type = FloatPairU; };
template <> struct PairU<double> { using type = DoublePairU; };

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }

// cos(2 pi k / 32), k in [0, 32) (correctly rounded decimal expansions for k <= 8)
__host__ __device__ constexpr double cos32_first_octant(int k) {
  return k == 0 ? 1.0
       : k == 1 ? 0.9807852804032304491261822
       : k == 2 ? 0.9238795325112867561281832
       : k == 3 ? 0.8314696123025452370787884
       : k == 4 ? 0.7071067811865475244008444
       : k == 5 ? 0.5555702330196022247428308
       : k == 6 ? 0.38268343236508977172846
       : k == 7 ? 0.1950903220161282678482849
       : 0.0;
}
__host__ __device__ constexpr double cos32(int k) {
  return k <= 8 ? cos32_first_octant(k)
       : (k <= 16 ? -cos32_first_octant(16 - k)
       : (k <= 24 ? -cos32_first_octant(k - 16) : cos32_first_octant(32 - k)));
}
__host__ __device__ constexpr double sin32(int k) { return cos32((k + 24) & 31); }

// z * exp(-2 pi i j / len), len a power of two <= 32, j < len; branches fold at compile time
template <typename T>
__device__ __forceinline__ cx<T> twiddle_const(cx<T> z, int j, int len) {
  const int k = j * (32 / len);  // angle = 2 pi k / 32
  if (k == 0) return z;
  if (k == 8) return {z.im, -z.re};                         // * (-i)
  if (k == 16) return {-z.re, -z.im};                       // * (-1)
  if (k == 24) return {-z.im, z.re};                        // * (+i)
  const T c = (T)cos32(k), s = (T)sin32(k);                 // w = c - i s
  if (k == 4) { const T h = c; return {h * (z.re + z.im), h * (z.im - z.re)}; }
  if (k == 12) { const T h = s; return {h * (z.im - z.re), -h * (z.re + z.im)}; }
  return {z.re * c + z.im * s, z.im * c - z.re * s};
}

__host__ __device__ constexpr int bitrev(int x, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1) << (bits - 1 - i);
  return r;
}

// In-register forward DFT of R = 2^LOGR points: radix-2 decimation in
// frequency, then the bit-reversal permutation (free register renaming).
template <typename T, int LOGR>
__device__ __forceinline__ void dft_reg(cx<T>* v) {
  constexpr int R = 1 << LOGR;
#pragma unroll
  for (int len = R; len >= 2; len >>= 1) {
    const int half = len >> 1;
#pragma unroll
    for (int blk = 0; blk < R; blk += len) {
#pragma unroll
      for (int j = 0; j < half; ++j) {
        const cx<T> a = v[blk + j], b = v[blk + j + half];
        v[blk + j] = cadd(a, b);
        v[blk + j + half] = twiddle_const(csub(a, b), j, len);
      }
    }
  }
  cx<T> tmp[R];
#pragma unroll
  for (int k = 0; k < R; ++k) tmp[k] = v[bitrev(k, LOGR)];
#pragma unroll
  for (int k = 0; k < R; ++k) v[k] = tmp[k];
}

// LOGR: log2 of the largest radix (default: one butterfly of E points per thread
// per pass); with LOGR < LOGE each thread runs E / R butterflies per pass.
// FORCE_SPLIT: exchange real and imaginary parts separately even when N complex
// points fit in LDS (half the LDS, so two workgroups can share a CU).
// PAIRED: the paired layout of the last forward pass (see above).
// HALF: exchange through an LDS buffer of N/2 complex points, the lower half of the
// index space first, then the upper half.  Which half a point is written to and read
// from never depends on the thread (the top index bit comes from the butterfly block
// or from r), so each half moves as many b64 accesses as the full exchange, at twice
// the barriers and half the LDS: two workgroups share a CU, one's exchanges overlapping
// the other's arithmetic.
template <typename T, int LOGN, int NT_, int LOGE, int LOGR_ = LOGE, bool FORCE_SPLIT = false,
          bool PAIRED_ = false, bool HALF_ = false>
struct BlockFFT {
  static constexpr int N = 1 << LOGN;
  static constexpr int NT = NT_;
  static constexpr int E = 1 << LOGE;
  static constexpr int LOGRMAX = LOGR_;
  static_assert(N == NT * E, "N must equal threads * points per thread");
  static_assert(LOGR_ <= LOGE, "radix larger than the points of a thread");
  static constexpr int P = LOGN / LOGR_;
  static constexpr int REM = LOGN % LOGR_;
  static constexpr int NP = P + (REM ? 1 : 0);
  // forward sequence: the short pass first; inverse sequence: the short pass last,
  // so the last forward pass and the first inverse pass share one data layout
  static constexpr int flog(int p) { return (REM && p == 0) ? REM : LOGR_; }
  static constexpr int ilog(int p) { return (REM && p == NP - 1) ? REM : LOGR_; }

  static constexpr int kLdsLimit = 160 * 1024;
  static constexpr int cx_pad_log = (sizeof(T) == 4) ? 4 : 3;  // 128 B / (2 sizeof T)
  static constexpr int sc_pad_log = (sizeof(T) == 4) ? 5 : 4;  // 128 B / sizeof T
  static constexpr int cx_bytes = (N + (N >> cx_pad_log)) * 2 * (int)sizeof(T);
  static constexpr int sc_bytes = (N + (N >> sc_pad_log)) * (int)sizeof(T);
  static constexpr bool HALF = HALF_;
  static constexpr int half_bytes = (N / 2 + ((N / 2) >> cx_pad_log)) * 2 * (int)sizeof(T);
  static constexpr bool SPLIT = !HALF && (FORCE_SPLIT || cx_bytes > kLdsLimit);
  static constexpr bool PAIRED = PAIRED_;
  static_assert(!PAIRED || (NP >= 2 && (E >> LOGR_) % 2 == 0), "paired layout needs an even butterfly count");
  // is pass p of a sequence in the paired layout (last forward pass, first reversed pass)
  static constexpr bool pass_paired(bool fwd, int p) { return PAIRED && (fwd ? p == NP - 1 : p == 0); }
  static constexpr int LDS_BYTES = HALF ? half_bytes : (SPLIT ? sc_bytes : cx_bytes);
  static_assert(!HALF || (NT * (1 << LOGR_) <= N / 2 && (1 << LOGR_) >= 2 && (LOGN % LOGR_ == 0 || (1 << (LOGN % LOGR_)) >= 2)),
                "half exchanges need at least two butterflies per thread");
  static_assert(!HALF || !PAIRED || (E >> LOGR_) == 2, "half exchanges with the paired layout need two butterflies");
  static_assert(LDS_BYTES <= kLdsLimit, "transform does not fit in LDS");

  __device__ static __forceinline__ int cpad(int i) { return i + (i >> cx_pad_log); }
  __device__ static __forceinline__ int spad(int i) { return i + (i >> sc_pad_log); }

  // butterfly handled as the i-th of thread t in a pass (PAIR: paired layout)
  template <bool PAIR>
  __device__ static __forceinline__ int bfly(int t, int i) {
    if constexpr (PAIR) {
      constexpr int NB = E >> LOGR_;   // butterflies per thread in the paired passes
      if (i % 2 == 0) return t + i * NT;
      return t == 0 ? i * NT : (NB - i + 1) * NT - t;
    } else {
      return t + i * NT;
    }
  }
  // output position of element (i, r) of thread t after a pass (LOGR, LOGNS)
  template <int LOGR, int LOGNS, bool PAIR = false>
  __device__ static __forceinline__ int out_index(int t, int i, int r) {
    const int b = bfly<PAIR>(t, i);
    return ((b >> LOGNS) << (LOGNS + LOGR)) + (b & ((1 << LOGNS) - 1)) + (r << LOGNS);
  }
  // input position of element (i, r) of thread t for a pass of radix 2^LOGR
  template <int LOGR, bool PAIR = false>
  __device__ static __forceinline__ int in_index(int t, int i, int r) {
    return bfly<PAIR>(t, i) + (r << (LOGN - LOGR));
  }
  // out_index(t, i, r) = out_base(t, i) + (r << LOGNS)
  template <int LOGR, int LOGNS, bool PAIR>
  __device__ static __forceinline__ int out_base(int t, int i) {
    const int b = bfly<PAIR>(t, i);
    return ((b >> LOGNS) << (LOGNS + LOGR)) + (b & ((1 << LOGNS) - 1));
  }
  // Index half (0: below N/2) of the output slot of element (i, r) of a pass (LOGR, LOGNS),
  // and of the input slot of element (i, r) of a pass of radix 2^LOGR2, for every thread.
  // Output: below the last pass the top bit is the top bit of the butterfly b < N/R,
  // i.e. of its block i NT (t < NT <= N/(2R)); the paired layout's odd i own block
  // NB - i = i (NB = 2).  In the last pass (Ns R = N) it is the top bit of r.  Input:
  // b < N/R2, so the top bit of b + r N/R2 is that of r.
  template <int LOGR, int LOGNS>
  static constexpr int out_half(int i, int r) {
    if constexpr (LOGNS + LOGR >= LOGN) {
      return r >> (LOGR - 1);
    } else {
      return (i * NT) >> (LOGN - LOGR - 1);
    }
  }
  template <int LOGR2>
  static constexpr int in_half(int r) { return r >> (LOGR2 - 1); }

  // Padded LDS slot of v + (r << LOGC), with the padding of the constant part
  // folded at compile time: v + c and v stay in rows (of 2^PL elements) that
  // differ by exactly floor(c / 2^PL) for every index an exchange forms.  Reads
  // have v = b, c = r N/R': c is a multiple of 2^PL, or v < N/R' divides 2^PL.
  // Writes have v = M + (b mod Ns), c = r Ns < Ns R with M a multiple of Ns R,
  // so (v + c) mod 2^PL never wraps past the row of v.
  template <int PL, int LOGC>
  __device__ static __forceinline__ int padded(int v, int r) {
    const int c = r << LOGC;
    return v + (v >> PL) + c + (c >> PL);
  }

  // ---- per-pass twiddle tables
  static constexpr int log_radix(bool fwd, int p) { return fwd ? flog(p) : ilog(p); }
  static constexpr int log_span(bool fwd, int p) {
    int s = 0;
    for (int q = 0; q < p; ++q) s += log_radix(fwd, q);
    return s;
  }
  static constexpr int tw_count(bool fwd, int p) {
    return log_span(fwd, p) == 0 ? 0 : (1 << (log_span(fwd, p) + log_radix(fwd, p)));
  }
  static constexpr int tw_total_seq(bool fwd) {
    int o = 0;
    for (int q = 0; q < NP; ++q) o += tw_count(fwd, q);
    return o;
  }
  static constexpr int tw_offset(bool fwd, int p) {
    int o = fwd ? 0 : tw_total_seq(true);
    for (int q = 0; q < p; ++q) o += tw_count(fwd, q);
    return o;
  }
  static constexpr int tw_total() { return tw_total_seq(true) + tw_total_seq(false); }

  // butterflies of one pass, in registers; ptab = this pass's table (rows of R factors)
  template <int LOGR, int LOGNS, bool PAIR>
  __device__ static __forceinline__ void butterflies(cx<T>* v, const cx<T>* __restrict__ ptab, int t) {
    constexpr int R = 1 << LOGR;
    constexpr int NB = E / R;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      if (LOGNS > 0) {
        const int j = bfly<PAIR>(t, i) & ((1 << LOGNS) - 1);
        const cx<T>* __restrict__ w = ptab + (j << LOGR);
#pragma unroll
        for (int r = 1; r < R; ++r) v[i * R + r] = cmul(v[i * R + r], w[r]);
      }
      dft_reg<T, LOGR>(v + i * R);
    }
  }

  // redistribute: element (i, r) of a pass (LOGR, LOGNS) goes to the slot of the next pass (LOGR2)
  template <int LOGR, int LOGNS, int LOGR2, bool PAIR_OUT, bool PAIR_IN>
  __device__ static __forceinline__ void exchange(cx<T>* v, void* lds_raw, int t) {
    constexpr int R = 1 << LOGR, NB = E / R;
    constexpr int R2 = 1 << LOGR2, NB2 = E / R2;
    if constexpr (HALF) {
      // the points read in the first half land in nv, not in v, whose upper-half points
      // are still to be written (the registers freed by the first writes take them)
      cx<T>* lds = reinterpret_cast<cx<T>*>(lds_raw);
      constexpr int HP = N / 2 + ((N / 2) >> cx_pad_log);   // padded slot of N/2
      cx<T> nv[E];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const int vb = out_base<LOGR, LOGNS, PAIR_OUT>(t, i);
#pragma unroll
          for (int r = 0; r < R; ++r)
            if (out_half<LOGR, LOGNS>(i, r) == h) lds[padded<cx_pad_log, LOGNS>(vb, r) - h * HP] = v[i * R + r];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NB2; ++i) {
          const int vb = bfly<PAIR_IN>(t, i);
#pragma unroll
          for (int r = 0; r < R2; ++r)
            if (in_half<LOGR2>(r) == h) nv[i * R2 + r] = lds[padded<cx_pad_log, LOGN - LOGR2>(vb, r) - h * HP];
        }
      }
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = nv[e];
    } else if constexpr (!SPLIT) {
      cx<T>* lds = reinterpret_cast<cx<T>*>(lds_raw);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int vb = out_base<LOGR, LOGNS, PAIR_OUT>(t, i);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[padded<cx_pad_log, LOGNS>(vb, r)] = v[i * R + r];
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < NB2; ++i) {
        const int vb = bfly<PAIR_IN>(t, i);
#pragma unroll
        for (int r = 0; r < R2; ++r) v[i * R2 + r] = lds[padded<cx_pad_log, LOGN - LOGR2>(vb, r)];
      }
    } else {
      T* lds = reinterpret_cast<T*>(lds_raw);
      // real parts, then imaginary parts; a component can be overwritten as soon as
      // the whole workgroup has stored it
#pragma unroll
      for (int part = 0; part < 2; ++part) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const int vb = out_base<LOGR, LOGNS, PAIR_OUT>(t, i);
#pragma unroll
          for (int r = 0; r < R; ++r)
            lds[padded<sc_pad_log, LOGNS>(vb, r)] = part ? v[i * R + r].im : v[i * R + r].re;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NB2; ++i) {
          const int vb = bfly<PAIR_IN>(t, i);
#pragma unroll
          for (int r = 0; r < R2; ++r) {
            const T x = lds[padded<sc_pad_log, LOGN - LOGR2>(vb, r)];
            if (part) v[i * R2 + r].im = x; else v[i * R2 + r].re = x;
          }
        }
      }
    }
  }

  // pass p of a sequence (FWD: forward order of radices, else inverse order)
  template <bool FWD, int p, int LOGNS>
  __device__ static __forceinline__ void run_from(cx<T>* v, void* lds, const cx<T>* __restrict__ ptw,
                                                  int t) {
    constexpr int LR = FWD ? flog(p) : ilog(p);
    constexpr bool PO = pass_paired(FWD, p);
    butterflies<LR, LOGNS, PO>(v, ptw + tw_offset(FWD, p), t);
    if constexpr (p + 1 < NP) {
      constexpr int LR2 = FWD ? flog(p + 1) : ilog(p + 1);
      exchange<LR, LOGNS, LR2, PO, pass_paired(FWD, p + 1)>(v, lds, t);
      run_from<FWD, p + 1, LOGNS + LR>(v, lds, ptw, t);
    }
  }

  // Input: point (i, r) of thread t holds x[in_index<first radix>(t, i, r)].
  // Output: point (i, r) holds X[fwd_out_index(t, i, r)] (forward DFT, no scaling).
  // ptw: the per-pass twiddle tables of this shape (tw_total() entries).
  __device__ static __forceinline__ void forward(cx<T>* v, void* lds, const cx<T>* __restrict__ ptw,
                                                 int t) {
    run_from<true, 0, 0>(v, lds, ptw, t);
  }
  // Same transform with the radix order reversed (first pass = forward's last radix);
  // its input layout is the forward output layout, its output point (i, r) holds
  // X[t + i NT + r N / R_last] with R_last its last radix.
  __device__ static __forceinline__ void forward_rev(cx<T>* v, void* lds, const cx<T>* __restrict__ ptw,
                                                     int t) {
    run_from<false, 0, 0>(v, lds, ptw, t);
  }

  // position of point (i, r) of thread t after forward()
  __device__ static __forceinline__ int fwd_out_index(int t, int i, int r) {
    return bfly<PAIRED>(t, i) + (r << (LOGN - flog(NP - 1)));
  }

  static constexpr int first_log_fwd() { return flog(0); }
  static constexpr int last_log_fwd() { return flog(NP - 1); }
  static constexpr int first_log_rev() { return ilog(0); }
  static constexpr int last_log_rev() { return ilog(NP - 1); }
};

}  // namespace mm
