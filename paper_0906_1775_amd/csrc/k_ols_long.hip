// Overlap-save N^-1 with transforms longer than one workgroup's registers and LDS
// (n_f = 2^17 and 2^18: the lengths of the paper's FFT-length rule for n_c = 8192,
// Weighting section, eqs. FFTcomplexity and FFTcomplexityFunction).
//
// The n_f = 2N real window is packed as N = N1 x N2 complex points z_n (as in the
// on-chip kernel) and transformed by the four-step decomposition, n = N2 n1 + n2,
// k = k1 + N1 k2:
//   X[k1 + N1 k2] = sum_n2 W_N2^(n2 k2) [ W_N^(n2 k1) sum_n1 z[N2 n1 + n2] W_N1^(n1 k1) ],
// in three kernels over a batch of (chunk, RHS) jobs whose N-point intermediates
// stay in device memory (sized so that a batch fits the last-level cache):
//   columns  N1-point transforms of the N2 columns (16 per workgroup, staged through
//            LDS so that every global access covers 16 consecutive points), times
//            W_N^(n2 k1), stored as rows Y[k1][n2];
//   rows     N2-point transforms of rows k1 and N1 - k1 (one wavefront each), the
//            real-to-complex pairing of X_k with X_(N-k) (row k1 element k2 pairs
//            with row N1 - k1 element N2 - 1 - k2; row 0 with itself, k2 with
//            N2 - k2), the filter symbol and the folding back to the packed output
//            spectrum (conjugated, as in the on-chip kernel), then the N2-point
//            transforms of the inverse's first step, times W_N^(k1 n2), in place;
//   output   N1-point transforms of the columns, and the valid outputs (the real and
//            negated imaginary parts, i.e. the conjugate) written back.
// The inverse transform is conj(FFT(conj Z')) with the same decomposition read the
// other way (input index k = k1 + N1 k2, output index n = N2 n1 + n2), and the 1/N
// of the inverse and the pairing's halvings are in the symbol table F/(4N).
#include <algorithm>

#include "fft.hpp"
#include "mm_internal.h"

namespace mm {

namespace {

// One sub-transform of 2^L points per wavefront: 64 threads x 4 (L = 8, radix-4 passes)
// or x 8 (L = 9, radix-8 passes) points; its per-pass twiddle tables are those of the
// on-chip transform of the same length (launch_pass_twiddles(L, ..., 0)).
template <int L> struct SubShape;
template <> struct SubShape<8> { static constexpr int LOGE = 2; };
template <> struct SubShape<9> { static constexpr int LOGE = 3; };
template <typename T, int L>
using SubFFT = BlockFFT<T, L, 64, SubShape<L>::LOGE, SubShape<L>::LOGE>;

constexpr int kL1 = 8;     // columns are 2^8-point transforms
constexpr int kCW = 16;    // columns per workgroup of the column kernels

template <typename V> struct Pair2;
template <> struct Pair2<float> { using type = float2; };
template <> struct Pair2<double> { using type = double2; };

// Tables of the four-step transform (LongTables): lo[j] = W_N^j (j < N2), hi[j] = W_N^(N2 j)
// (j < N1), so W_N^j = hi[j / N2] lo[j mod N2] for j < N; r2[k2] = exp(-2 pi i k2 / (2 N2))
// (k2 < N2), so the pairing's exp(-2 pi i k / (2N)) at k = k1 + N1 k2 is tw2[k1] r2[k2].
template <typename T, int L1, int L2>
struct LongTables {
  static constexpr int N1 = 1 << L1, N2 = 1 << L2;
  static constexpr int LO = 0, HI = N2, R2 = N2 + N1, TOTAL = 2 * N2 + N1;
};

template <typename T, int L1, int L2>
__device__ __forceinline__ cx<T> w_n(const cx<T>* __restrict__ tab, int j) {
  using LT = LongTables<T, L1, L2>;
  return cmul(tab[LT::HI + (j >> L2)], tab[LT::LO + (j & (LT::N2 - 1))]);
}

template <typename T, int L1, int L2>
constexpr int col_lds_bytes() {
  constexpr int a = 16 * SubFFT<T, L1>::LDS_BYTES;
  constexpr int b = kCW * ((1 << L1) + 1) * (int)sizeof(cx<T>);
  constexpr int c = (1 << L1) * (kCW + 1) * (int)sizeof(cx<T>);
  return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

}  // namespace

// columns of the forward transform: work[j][k1][n2] = W_N^(n2 k1) sum_n1 z[N2 n1 + n2] W_N1^(n1 k1)
template <typename T, typename Tin, int L1, int L2>
__global__ __launch_bounds__(1024) void k_long_columns(const Tin* __restrict__ yin, cx<T>* __restrict__ work,
                                                       const OlsChunk* __restrict__ chunks, int64_t job0,
                                                       int n_chunks, int64_t n_t, int n_c,
                                                       const CgState* __restrict__ st,
                                                       const cx<T>* __restrict__ ptw1,
                                                       const cx<T>* __restrict__ ltab) {
  using F1 = SubFFT<T, L1>;
  constexpr int N1 = 1 << L1, N2 = 1 << L2, NG = N2 / kCW, TS = N1 + 1, OS = kCW + 1;
  constexpr int64_t N = (int64_t)N1 * N2;
  __shared__ __align__(16) char lds[col_lds_bytes<T, L1, L2>()];
  const int64_t jl = blockIdx.x / NG;
  const int cg = blockIdx.x % NG;
  const int64_t job = job0 + jl;
  const int rhs = (int)(job / n_chunks);
  if (st && !st[rhs].active) return;   // this RHS has stopped iterating
  const OlsChunk ch = chunks[job - (int64_t)rhs * n_chunks];
  const Tin* __restrict__ src = yin + (int64_t)rhs * n_t;
  const int64_t s0 = ch.out_start - n_c, lo = ch.iv_lo, hi = ch.iv_hi;
  cx<T>* tile = reinterpret_cast<cx<T>*>(lds);
  const int tid = threadIdx.x;
  // the workgroup's 16 columns, row by row: 16 consecutive points = 32 consecutive samples
#pragma unroll
  for (int q = 0; q < N1 * kCW / 1024; ++q) {
    const int e = tid + 1024 * q;
    const int c = e % kCW, n1 = e / kCW;
    const int64_t j = s0 + 2 * ((int64_t)N2 * n1 + cg * kCW + c);
    const T a = (j >= lo && j < hi) ? (T)src[j] : (T)0;
    const T b = (j + 1 >= lo && j + 1 < hi) ? (T)src[j + 1] : (T)0;
    tile[c * TS + n1] = {a, b};
  }
  __syncthreads();
  const int w = tid >> 6, t = tid & 63;   // wavefront w transforms column cg * 16 + w
  cx<T> v[F1::E];
#pragma unroll
  for (int r = 0; r < F1::E; ++r) v[r] = tile[w * TS + t + 64 * r];
  // (the transform's first exchange begins with a barrier: every column is in registers
  // before any wavefront reuses the tile's LDS)
  F1::forward(v, lds + w * F1::LDS_BYTES, ptw1, t);
  const int n2 = cg * kCW + w;
#pragma unroll
  for (int r = 0; r < F1::E; ++r) v[r] = cmul(v[r], w_n<T, L1, L2>(ltab, n2 * (t + 64 * r)));   // n2 k1 < N
  __syncthreads();
#pragma unroll
  for (int r = 0; r < F1::E; ++r) tile[(t + 64 * r) * OS + w] = v[r];
  __syncthreads();
  cx<T>* __restrict__ dst = work + jl * N;
#pragma unroll
  for (int q = 0; q < N1 * kCW / 1024; ++q) {
    const int e = tid + 1024 * q;
    const int c = e % kCW, k1 = e / kCW;
    dst[(int64_t)k1 * N2 + cg * kCW + c] = tile[k1 * OS + c];
  }
}

// rows k1 = g and N1 - g: forward N2-point transforms, pairing and symbol, then the
// first step of the inverse (N2-point transforms, times W_N^(k1 n2)), in place
template <typename T, int L1, int L2>
__global__ __launch_bounds__(128) void k_long_rows(cx<T>* __restrict__ work, const OlsChunk* __restrict__ chunks,
                                                   int64_t job0, int n_chunks, const CgState* __restrict__ st,
                                                   const T* __restrict__ spec_rows, const cx<T>* __restrict__ ptw2,
                                                   const cx<T>* __restrict__ tw2, const cx<T>* __restrict__ ltab) {
  using F2 = SubFFT<T, L2>;
  constexpr int N1 = 1 << L1, N2 = 1 << L2, NP = N1 / 2 + 1;
  constexpr int64_t N = (int64_t)N1 * N2;
  __shared__ __align__(16) char lds[2 * F2::LDS_BYTES];
  __shared__ cx<T> spx[2][N2];
  const int64_t jl = blockIdx.x / NP;
  const int g = blockIdx.x % NP;
  const int64_t job = job0 + jl;
  const int rhs = (int)(job / n_chunks);
  if (st && !st[rhs].active) return;   // this RHS has stopped iterating
  const OlsChunk ch = chunks[job - (int64_t)rhs * n_chunks];
  const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int a = g, b = (N1 - g) & (N1 - 1);   // a = b for rows 0 and N1/2 (both wavefronts hold it)
  const int row = w == 0 ? a : b;
  cx<T>* __restrict__ base = work + jl * N;
  cx<T> v[F2::E];
#pragma unroll
  for (int r = 0; r < F2::E; ++r) v[r] = base[(int64_t)row * N2 + t + 64 * r];
  F2::forward(v, lds + w * F2::LDS_BYTES, ptw2, t);
  // v[r] = X[row + N1 k2], k2 = t + 64 r
#pragma unroll
  for (int r = 0; r < F2::E; ++r) spx[w][t + 64 * r] = v[r];
  __syncthreads();
  // For the pair (k, N-k): A = X_k, B = conj X_(N-k), E = A + B, O = -i (A - B),
  // Y = (E + W O) F_k, Y' = (E - W O) F_(N-k), W = e^(-2 pi i k/(2N)); the transform of
  // the inverse's input at k is conj(s + i W^-1 d), s = Y + Y', d = Y - Y'.
  // the symbol in row order: SR[k1 N2 + k2] = F_(k1 + N1 k2) / (4N), SR[N] = F_N / (4N)
  const T* __restrict__ SR = spec_rows + (int64_t)ch.filter * (N + 1);
  using LT = LongTables<T, L1, L2>;
  const cx<T> wrow = tw2[row];
#pragma unroll
  for (int r = 0; r < F2::E; ++r) {
    const int k2 = t + 64 * r;
    const cx<T> partner = row == 0 ? spx[w][(N2 - k2) & (N2 - 1)] : spx[1 - w][N2 - 1 - k2];
    const cx<T> A = v[r];
    const cx<T> B = cconj(partner);
    const cx<T> Ev = cadd(A, B);
    const cx<T> D = csub(A, B);
    const cx<T> O = {D.im, -D.re};
    const cx<T> W = cmul(wrow, ltab[LT::R2 + k2]);   // exp(-2 pi i k / (2N)), k = row + N1 k2
    const cx<T> WO = cmul(W, O);
    // F_(N-k): row N1 - row, element N2 - 1 - k2 (row 0: element N2 - k2, and F_N for k2 = 0)
    const T sa = SR[(int64_t)row * N2 + k2];
    const T sb = row != 0 ? SR[(int64_t)(N1 - row) * N2 + (N2 - 1 - k2)] : (k2 == 0 ? SR[N] : SR[N2 - k2]);
    const cx<T> Y = cscale(cadd(Ev, WO), sa);
    const cx<T> Yp = cscale(csub(Ev, WO), sb);
    const cx<T> sum = cadd(Y, Yp);
    const cx<T> Wd = cmul(cconj(W), csub(Y, Yp));
    v[r] = {sum.re - Wd.im, -(sum.im + Wd.re)};
  }
  F2::forward(v, lds + w * F2::LDS_BYTES, ptw2, t);
  if (a == b && w == 1) return;   // the second copy of a row paired with itself
#pragma unroll
  for (int r = 0; r < F2::E; ++r) {
    const int n2 = t + 64 * r;
    base[(int64_t)row * N2 + n2] = cmul(v[r], w_n<T, L1, L2>(ltab, row * n2));   // row n2 < N
  }
}

// columns of the inverse: N1-point transforms over k1, conjugated, and the valid outputs
template <typename T, int L1, int L2>
__global__ __launch_bounds__(1024) void k_long_output(const cx<T>* __restrict__ work, T* __restrict__ yout,
                                                      const OlsChunk* __restrict__ chunks, int64_t job0,
                                                      int n_chunks, int64_t n_t, int n_c, int m,
                                                      const CgState* __restrict__ st,
                                                      const cx<T>* __restrict__ ptw1) {
  using F1 = SubFFT<T, L1>;
  constexpr int N1 = 1 << L1, N2 = 1 << L2, NG = N2 / kCW, TS = N1 + 1, OS = kCW + 1;
  constexpr int64_t N = (int64_t)N1 * N2;
  __shared__ __align__(16) char lds[col_lds_bytes<T, L1, L2>()];
  const int64_t jl = blockIdx.x / NG;
  const int cg = blockIdx.x % NG;
  const int64_t job = job0 + jl;
  const int rhs = (int)(job / n_chunks);
  if (st && !st[rhs].active) return;   // this RHS has stopped iterating
  const OlsChunk ch = chunks[job - (int64_t)rhs * n_chunks];
  const int64_t s0 = ch.out_start - n_c, hi = ch.iv_hi;
  cx<T>* tile = reinterpret_cast<cx<T>*>(lds);
  const int tid = threadIdx.x;
  const cx<T>* __restrict__ srcw = work + jl * N;
#pragma unroll
  for (int q = 0; q < N1 * kCW / 1024; ++q) {
    const int e = tid + 1024 * q;
    const int c = e % kCW, k1 = e / kCW;
    tile[c * TS + k1] = srcw[(int64_t)k1 * N2 + cg * kCW + c];
  }
  __syncthreads();
  const int w = tid >> 6, t = tid & 63;
  cx<T> v[F1::E];
#pragma unroll
  for (int r = 0; r < F1::E; ++r) v[r] = tile[w * TS + t + 64 * r];
  F1::forward(v, lds + w * F1::LDS_BYTES, ptw1, t);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < F1::E; ++r) tile[(t + 64 * r) * OS + w] = v[r];   // output n1 = t + 64 r
  __syncthreads();
  T* __restrict__ dst = yout + (int64_t)rhs * n_t;
#pragma unroll
  for (int q = 0; q < N1 * kCW / 1024; ++q) {
    const int e = tid + 1024 * q;
    const int c = e % kCW, n1 = e / kCW;
    const int64_t pos = 2 * ((int64_t)N2 * n1 + cg * kCW + c);
    const cx<T> z = tile[n1 * OS + c];
    if (pos >= n_c && pos < n_c + m && s0 + pos < hi) dst[s0 + pos] = z.re;
    if (pos + 1 >= n_c && pos + 1 < n_c + m && s0 + pos + 1 < hi) dst[s0 + pos + 1] = -z.im;
  }
}

// LongTables of a transform of 2^logn points, from float64 angles
template <typename T, int L1, int L2>
__global__ void k_long_tables(cx<T>* __restrict__ tab) {
  using LT = LongTables<T, L1, L2>;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= LT::TOTAL) return;
  double frac;   // angle / (-2 pi)
  if (e < LT::HI) frac = (double)e / (double)(LT::N1 * LT::N2);
  else if (e < LT::R2) frac = (double)(e - LT::HI) / (double)LT::N1;
  else frac = (double)(e - LT::R2) / (double)(2 * LT::N2);
  double sn, cs;
  sincospi(2.0 * frac, &sn, &cs);
  tab[e] = {(T)cs, (T)(-sn)};
}

// spec_rows[f][k1 N2 + k2] = spec[f][k1 + N1 k2], spec_rows[f][N] = spec[f][N]
template <typename T, int L1, int L2>
__global__ void k_long_symbol_rows(const T* __restrict__ spec, T* __restrict__ rows) {
  constexpr int N1 = 1 << L1, N2 = 1 << L2;
  constexpr int64_t N = (int64_t)N1 * N2;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e > N) return;
  const T* __restrict__ src = spec + (int64_t)blockIdx.y * (N + 1);
  T* __restrict__ dst = rows + (int64_t)blockIdx.y * (N + 1);
  dst[e] = e == N ? src[N] : src[(e & (N2 - 1)) * N1 + (e >> L2)];
}

int ols_long_table_count(int logn) { return 2 * (1 << (logn - kL1)) + (1 << kL1); }

template <typename T, int L2>
static hipError_t long_tables_launch(void* tab, hipStream_t s) {
  using LT = LongTables<T, kL1, L2>;
  hipLaunchKernelGGL((k_long_tables<T, kL1, L2>), dim3((LT::TOTAL + 255) / 256), dim3(256), 0, s, (cx<T>*)tab);
  return hipGetLastError();
}

template <typename T, int L2>
static hipError_t symbol_rows_launch(const void* spec, void* rows, int n_filters, hipStream_t s) {
  if (n_filters <= 0) return hipSuccess;
  const int64_t n = (int64_t(1) << (kL1 + L2)) + 1;
  hipLaunchKernelGGL((k_long_symbol_rows<T, kL1, L2>), dim3((unsigned)((n + 255) / 256), (unsigned)n_filters),
                     dim3(256), 0, s, (const T*)spec, (T*)rows);
  return hipGetLastError();
}

hipError_t launch_long_tables(int logn, bool fp64, void* tab, hipStream_t s) {
  if (logn == kL1 + 8) return fp64 ? long_tables_launch<double, 8>(tab, s) : long_tables_launch<float, 8>(tab, s);
  if (logn == kL1 + 9) return fp64 ? long_tables_launch<double, 9>(tab, s) : long_tables_launch<float, 9>(tab, s);
  return hipErrorInvalidValue;
}

hipError_t launch_long_symbol_rows(int logn, bool fp64, const void* spec, void* rows, int n_filters, hipStream_t s) {
  if (logn == kL1 + 8)
    return fp64 ? symbol_rows_launch<double, 8>(spec, rows, n_filters, s)
                : symbol_rows_launch<float, 8>(spec, rows, n_filters, s);
  if (logn == kL1 + 9)
    return fp64 ? symbol_rows_launch<double, 9>(spec, rows, n_filters, s)
                : symbol_rows_launch<float, 9>(spec, rows, n_filters, s);
  return hipErrorInvalidValue;
}

bool ols_long_exists(int logn) { return logn == kL1 + 8 || logn == kL1 + 9; }

int64_t ols_long_batch(int logn, bool fp64) {
  const int64_t job_bytes = (int64_t(1) << logn) * (fp64 ? 16 : 8);
  return std::max<int64_t>(1, (int64_t(64) << 20) / job_bytes);
}

template <typename T, typename Tin, int L2>
static hipError_t long_launch(const void* y_in, void* y_out, const OlsChunk* chunks, int n_chunks, const void* spec,
                              const void* ptw1, const void* ptw2, const void* tw2, const void* ltab, void* work,
                              int64_t batch, int64_t n_t, int n_c, int m, int n_rhs, hipStream_t s,
                              const CgState* st) {
  constexpr int NG = (1 << L2) / kCW, NP = (1 << kL1) / 2 + 1;
  const int64_t n_jobs = (int64_t)n_chunks * n_rhs;
  for (int64_t j0 = 0; j0 < n_jobs; j0 += batch) {
    const int64_t nb = std::min(batch, n_jobs - j0);
    hipLaunchKernelGGL((k_long_columns<T, Tin, kL1, L2>), dim3((unsigned)(nb * NG)), dim3(1024), 0, s,
                       (const Tin*)y_in, (cx<T>*)work, chunks, j0, n_chunks, n_t, n_c, st, (const cx<T>*)ptw1,
                       (const cx<T>*)ltab);
    hipLaunchKernelGGL((k_long_rows<T, kL1, L2>), dim3((unsigned)(nb * NP)), dim3(128), 0, s, (cx<T>*)work, chunks,
                       j0, n_chunks, st, (const T*)spec, (const cx<T>*)ptw2, (const cx<T>*)tw2,
                       (const cx<T>*)ltab);
    hipLaunchKernelGGL((k_long_output<T, kL1, L2>), dim3((unsigned)(nb * NG)), dim3(1024), 0, s,
                       (const cx<T>*)work, (T*)y_out, chunks, j0, n_chunks, n_t, n_c, m, st, (const cx<T>*)ptw1);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T, typename Tin>
static hipError_t long_dispatch(int logn, const void* y_in, void* y_out, const OlsChunk* chunks, int n_chunks,
                                const void* spec, const void* ptw1, const void* ptw2, const void* tw2,
                                const void* ltab, void* work, int64_t batch, int64_t n_t, int n_c, int m, int n_rhs,
                                hipStream_t s, const CgState* st) {
  if (logn == kL1 + 8)
    return long_launch<T, Tin, 8>(y_in, y_out, chunks, n_chunks, spec, ptw1, ptw2, tw2, ltab, work, batch, n_t, n_c,
                                  m, n_rhs, s, st);
  if (logn == kL1 + 9)
    return long_launch<T, Tin, 9>(y_in, y_out, chunks, n_chunks, spec, ptw1, ptw2, tw2, ltab, work, batch, n_t, n_c,
                                  m, n_rhs, s, st);
  return hipErrorInvalidValue;
}

hipError_t launch_ols_long(bool fp64, bool in_f64, int logn, const void* y_in, void* y_out, const OlsChunk* chunks,
                           int n_chunks, const void* spec_rows, const void* ptw1, const void* ptw2, const void* tw2,
                           const void* ltab, void* work, int64_t batch, int64_t n_t, int n_c, int m, int n_rhs,
                           hipStream_t s, const CgState* st) {
  if (n_chunks == 0 || n_rhs == 0) return hipSuccess;
  if (batch < 1) return hipErrorInvalidValue;
  if (fp64)
    return in_f64 ? long_dispatch<double, double>(logn, y_in, y_out, chunks, n_chunks, spec_rows, ptw1, ptw2, tw2,
                                                  ltab, work, batch, n_t, n_c, m, n_rhs, s, st)
                  : long_dispatch<double, float>(logn, y_in, y_out, chunks, n_chunks, spec_rows, ptw1, ptw2, tw2,
                                                 ltab, work, batch, n_t, n_c, m, n_rhs, s, st);
  return in_f64 ? long_dispatch<float, double>(logn, y_in, y_out, chunks, n_chunks, spec_rows, ptw1, ptw2, tw2, ltab,
                                               work, batch, n_t, n_c, m, n_rhs, s, st)
                : long_dispatch<float, float>(logn, y_in, y_out, chunks, n_chunks, spec_rows, ptw1, ptw2, tw2, ltab,
                                              work, batch, n_t, n_c, m, n_rhs, s, st);
}

}  // namespace mm
