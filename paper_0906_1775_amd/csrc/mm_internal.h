// Internal declarations shared by the host library and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mm {

// One overlap-save transform: outputs [out_start, min(out_start + m, iv_hi)) of
// the interval [iv_lo, iv_hi); the transform input starts n_c samples earlier.
struct OlsChunk {
  int64_t out_start;
  int64_t iv_lo;
  int64_t iv_hi;
  int32_t filter;
  int32_t pad;
};

// Per-RHS conjugate-gradient scalars, resident in device memory.
struct CgState {
  double rho;        // r . z
  double alpha;
  double beta;
  double bnorm;      // ||b||_2
  double rel;        // ||r||_2 / ||b||_2 of the current iterate
  double best_rel;   // lowest relative residual so far
  double tol;
  int32_t iter;      // iterations performed while active
  int32_t best_iter;
  int32_t active;    // 1 while the RHS still iterates
  int32_t copy_best; // set when the current iterate became the best
  int32_t fixed;     // 1 = ignore tol
  int32_t breakdown; // set when p.q <= 0 (H not positive definite on p)
  int32_t xcur;      // buffer of the current iterate: 0 = x, 1 = x_best (float64 x only)
  int32_t xbest;     // buffer of the lowest-residual iterate; -1 = none kept (reliable updates)
};

// A run of samples [t0, t1) inside one HWP-template segment or one stationary
// interval (id = segment or interval index).
struct SampleTile {
  int64_t t0;
  int64_t t1;
  int32_t id;
  int32_t pad;
};

constexpr int kTileSamples = 4096;  // samples per SampleTile
constexpr int kHwpHarmonics = 8;    // harmonics k = 1..8 of the HWP template
constexpr int kHwpColumns = 32;     // its columns per segment
constexpr int kMaxRhs = 64;

constexpr int kDotBlocks = 256;     // partial sums per dot product (fixed => deterministic)
constexpr int kDotThreads = 256;
constexpr int kScatterBlocks = 2048; // bound on the scatter grid (and its p.q partial sums)

// sum over aligned groups of G lanes (G a power of two <= 64)
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

// ---------------------------------------------------------------- filter (k_filter.hip)
int ols_max_logn(bool fp64);
hipError_t launch_tw2_table(void* tw2, int logn, bool fp64, hipStream_t s);
// per-pass twiddle tables of the workgroup transform of 2^logn points
// (variant: workgroup shape of the overlap-save transform; 0 for every other use)
int pass_twiddle_count(int logn, bool fp64, int variant = 0);
hipError_t launch_pass_twiddles(void* tab, int logn, bool fp64, hipStream_t s, int variant = 0);
// whether the overlap-save transform of 2^logn points has workgroup shape `variant`
constexpr int kOlsVariants = 10;
bool ols_variant_exists(int logn, bool fp64, int variant);
// lags (mode 0) or their derivative with respect to sigma (1), f_knee (2), alpha (3)
hipError_t launch_lags(const double* params /*dev [nf][3]*/, int n_filters, double f_samp, int n_c,
                       int64_t lag_len, double* lags /*dev [nf][n_c]*/, void* scratch,
                       size_t scratch_bytes, hipStream_t s, int mode = 0);
size_t lags_scratch_bytes(int n_c, int64_t lag_len, int filters_per_batch);
// spec[f][k] = F_k / (4N), k = 0..N, the symbol of filter f's circulant of n_f = 2N points
size_t spectra_scratch_bytes(int logn);
hipError_t launch_spectra(const double* lags, int n_filters, int n_c, int logn, bool fp64,
                          void* spec /*[nf][N+1]*/, void* scratch, hipStream_t s);
// y_out[r][t] = (N^-1 y_in)[r][t]; compute type T (fp64 flag); input type in_f64; output type T
// st (optional): per-RHS CG states; rows of RHS no longer active are skipped
hipError_t launch_ols(bool fp64, bool in_f64, int logn, const void* y_in, void* y_out,
                      const OlsChunk* chunks, int n_chunks, const void* spec, const void* ptw,
                      const void* tw2, int64_t n_t, int n_c, int m, int n_rhs, hipStream_t s,
                      int variant = 0, const CgState* st = nullptr);

// ---------------------------------------------------------------- long filter (k_ols_long.hip)
// The overlap-save N^-1 with transforms of 2^logn complex points beyond one workgroup
// (logn 16 and 17, n_f = 2^17 and 2^18), as a batched four-step transform: ptw1 / ptw2 =
// launch_pass_twiddles tables of lengths 2^8 and 2^(logn - 8), tw2 as for launch_ols,
// work = device buffer of batch jobs x 2^logn complex points of the compute type.
// spec_rows: the symbol table in row order (launch_long_tables), ltab: its twiddle tables
// four-step transforms of 2^14 and 2^15 points (NO x 1024, NO = 16, 32) with wavefront-private
// inner stages (variant 9, float32): tab = its twiddle tables (ols_wave_table_count complex
// entries, launch_wave_tables); spec_w[f] = launch_spectra's table in row order (entry
// r * 1024 + k_in holds k = r + NO k_in, entry N holds k = N)
bool ols_wave_exists(int logn, bool fp64);
int ols_wave_table_count(int logn);
hipError_t launch_wave_tables(int logn, void* tab, hipStream_t s);
hipError_t launch_wave_symbols(int logn, const void* spec, void* spec_w, int n_filters, hipStream_t s);
hipError_t launch_ols_wave(int logn, bool in_f64, const void* y_in, void* y_out, const OlsChunk* chunks,
                           int n_chunks, const void* spec_w, const void* tab, int64_t n_t, int n_c, int m,
                           int n_rhs, hipStream_t s, const CgState* st);
bool ols_long_exists(int logn);
int64_t ols_long_batch(int logn, bool fp64);   // jobs per batch (intermediates of ~64 MiB)
int ols_long_table_count(int logn);            // complex entries of ltab
hipError_t launch_long_tables(int logn, bool fp64, void* ltab, hipStream_t s);
// spec_rows[f] = spec[f] (launch_spectra's tables) in row order: entry k1 N2 + k2 holds
// k = k1 + N1 k2 (N1 = 2^8, N2 = 2^(logn - 8)), entry N holds k = N; n_filters tables
hipError_t launch_long_symbol_rows(int logn, bool fp64, const void* spec, void* spec_rows, int n_filters,
                                   hipStream_t s);
hipError_t launch_ols_long(bool fp64, bool in_f64, int logn, const void* y_in, void* y_out, const OlsChunk* chunks,
                           int n_chunks, const void* spec_rows, const void* ptw1, const void* ptw2, const void* tw2,
                           const void* ltab, void* work, int64_t batch, int64_t n_t, int n_c, int m, int n_rhs,
                           hipStream_t s, const CgState* st = nullptr);

// ---------------------------------------------------------------- pointing (k_pointing.hip)
// y[r][t] = (P p_r)_t; p rows of stride vs (map values first, observed layout)
// p32 (optional): a float32 copy of the map part of p (rows of stride vs32), read
// instead of p; order (optional): the gather tiles (gather_tiles(n_t) runs of
// consecutive samples) in the order their blocks should run (sorted by pixel)
hipError_t launch_gather(bool out_f64, int ns, const int32_t* pix_obs, const float* w,
                         const double* p, int64_t vs, void* y, int64_t n_t, int64_t n_obs, int n_rhs,
                         hipStream_t s, const CgState* st = nullptr, const float* p32 = nullptr,
                         int64_t vs32 = 0, const int32_t* order = nullptr);
// runs of consecutive samples the gather assigns to one block
int64_t gather_tiles(int64_t n_t);
// key[i] = smallest observed id among the samples of gather tile i, -1 if none
hipError_t launch_tile_keys(const int32_t* pix_obs, int64_t n_t, int32_t* key, hipStream_t s);
// dst[r * dst_stride + i] = (float)src[r * src_stride + i], i < n
hipError_t launch_rows_to_f32(const double* src, int64_t src_stride, float* dst, int64_t dst_stride, int64_t n,
                              int n_rhs, hipStream_t s);
// Sliced pixel-major pointing (64 pixels per slice, one lane per pixel)
struct SellLayout {
  const uint32_t* end = nullptr;   // [n_slices] inclusive prefix sum of the slice sizes
  const uint32_t* len = nullptr;   // [n_slices] entries of each slice (64 x its widest pixel)
  const int32_t* t = nullptr;      // sample index per entry, -1 = padding
  const float* w = nullptr;        // (sin, cos) per entry (polarisation only)
  int wps = 8;                     // wavefronts per slice in the scatter (1, 2, 4 or 8); 0 = no
                                   // slices: one wavefront per pixel over the pixel-major arrays
  const int64_t* ptr = nullptr;    // pixel-major layout (wps = 0): [n_obs + 1] offsets,
  const int32_t* perm = nullptr;   // [n_valid] sample ids
  const float* w_pm = nullptr;     // [n_valid][2] (sin, cos) (polarisation only)
};
hipError_t launch_sell_widths(const int64_t* pix_ptr, int64_t n_obs, uint32_t* slice_len, hipStream_t s);
hipError_t launch_sell_fill(const int64_t* pix_ptr, const int32_t* perm, const float* w_pm, int64_t n_obs,
                            const uint32_t* slice_end, const uint32_t* slice_len, int32_t* sell_t,
                            float* sell_w, int ns, hipStream_t s);
// q = P^T y (observed layout, rows of stride vs).  When p is given, also
// pq_part[r * pq_stride + pq_slot + block] = partial sums of p.q over the pixels
// of each scatter block (scatter_blocks() blocks).
hipError_t launch_scatter(bool in_f64, int ns, const SellLayout& L, const void* y, double* q, int64_t vs,
                          int64_t n_obs, int64_t n_t, int n_rhs, hipStream_t s,
                          const double* p = nullptr, double* pq_part = nullptr, int pq_stride = 0,
                          int pq_slot = 0, const CgState* st = nullptr);
// The same with float32 y and q, and the p.q partial sums from the float32 copy of p
// (p32, rows of stride vs32): the mixed-precision iteration's scatter.
hipError_t launch_scatter_q32(int ns, const SellLayout& L, const float* y, float* q, int64_t vs, int64_t n_obs,
                              int64_t n_t, int n_rhs, hipStream_t s, const float* p32, int64_t vs32,
                              double* pq_part, int pq_stride, int pq_slot, const CgState* st);
// blocks (= p.q partial sums) of a scatter over n_obs pixels with wps wavefronts per slice
int scatter_blocks(int64_t n_obs, int wps);
int scatter_waves_per_slice(double avg_entries_per_pixel);   // 0: pixel-major, no slices
hipError_t launch_convert(bool in_f64, bool out_f64, const void* in, void* out, int64_t n,
                          hipStream_t s);
// observed <-> global layout of n_rhs rows (strides obs_stride, glob_stride in doubles)
hipError_t launch_to_observed(const double* glob, int64_t glob_stride, double* obs, int64_t obs_stride,
                              const int32_t* obs2glob, int64_t n_obs, int64_t n_pix, int ns, int n_rhs,
                              hipStream_t s);
hipError_t launch_to_global(const double* obs, int64_t obs_stride, double* glob, int64_t glob_stride,
                            const int32_t* obs2glob, int64_t n_obs, int64_t n_pix, int ns, int n_rhs,
                            hipStream_t s);
hipError_t launch_hits(const int64_t* pix_ptr, const int32_t* obs2glob, int32_t* hits,
                       int64_t n_obs, int64_t n_pix, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);

// ---------------------------------------------------------------- plan (k_sort.hip)
// flag[0] = 1 if any pix is < -1 or >= n_pix
hipError_t launch_check_pix(const int32_t* pix, int64_t n, int64_t n_pix, int32_t* flag,
                            hipStream_t s);
size_t sort_scratch_bytes(int64_t n);
// Stable sort of sample ids by pixel; excised samples (pix = -1) go last.
// keys_out[i] = pixel of the i-th sample in pixel-major order, vals_out[i] = its sample id.
hipError_t launch_sort_by_pixel(const int32_t* pix, int64_t n, int64_t n_pix, uint32_t* keys_out,
                                int32_t* vals_out, void* scratch, hipStream_t s);
size_t scan_scratch_bytes(int64_t n);
// inclusive scan of uint32 values
hipError_t launch_scan_inclusive(const uint32_t* in, uint32_t* out, int64_t n, void* scratch,
                                 hipStream_t s);
// flags[i] = 1 where a new pixel segment starts (i < n_valid)
// seg[i] = observed id + 1 of sorted sample i (runs of equal keys below n_pix counted
// up to i), and n_valid[0] = number of keys below n_pix (n_valid[0] must be 0
// beforehand); scratch of scan_scratch_bytes(n) bytes
hipError_t launch_segment_scan(const uint32_t* keys, int64_t n, uint32_t n_pix, uint32_t* seg, int64_t* n_valid,
                               void* scratch, hipStream_t s);
// pix_ptr, obs2glob, w_pm, perm from the sorted order
hipError_t launch_build_layout(const uint32_t* keys, const int32_t* vals, const uint32_t* seg_id,
                               int64_t n, uint32_t n_pix, const float* w, int ns, int64_t* pix_ptr,
                               int32_t* obs2glob, float* w_pm, int32_t* perm, hipStream_t s);
// time-major observed index pix_obs[t] (-1 for excised samples) through the inverse map
// glob2obs [n_keys] (scratch) of obs2glob; the keys must be in [-1, n_keys)
hipError_t launch_obs_index(const int32_t* key, int64_t n, const int32_t* obs2glob, int64_t n_obs,
                            int32_t* glob2obs, int64_t n_keys, int32_t* pix_obs, hipStream_t s);

// out[b] = sum over interval b of u_t v_t (one workgroup per interval, fixed order)
hipError_t launch_interval_dots(const double* u, const double* v, const int64_t* iv_start, int n_iv,
                                double* out, hipStream_t s);

// ---------------------------------------------------------------- CG (k_cg.hip)
// iv_hint[t >> hint_shift]: an interval starting at or before sample t, at most a few
// interval starts before the one that holds t
hipError_t launch_precond_build(int ns, int kind, int group, const int64_t* pix_ptr, const int32_t* perm,
                                const float* w_pm, const int64_t* iv_start, int n_iv, const int32_t* iv_hint,
                                int hint_shift, const int32_t* iv_filter, const double* lags, int n_c,
                                int64_t n_obs, double* minv, int32_t* singular, hipStream_t s);
// *out = number of nonzero flags[0..n) (out is cleared first; plan time only)
hipError_t launch_count_nonzero(const int32_t* flags, int64_t n, unsigned long long* out, hipStream_t s);
hipError_t launch_dot(const double* x, const double* y, int64_t nu, int n_rhs, double* partial,
                      hipStream_t s);
hipError_t launch_cg_init(CgState* st, const double* partial_bb, const double* partial_rr,
                          const double* partial_rz, double tol, int fixed, int n_rhs,
                          double* history, int hist_stride, hipStream_t s);
// r -= alpha q, z = M r with alpha = rho / (p.q) folded from the n_pq partial sums of
// p.q (x += alpha p is left to launch_cg_step_next); writes the r.z and r.r partial sums
// Vectors are rows of stride vs: n_obs pixel blocks, then n_tail template
// amplitudes preconditioned by the diagonal minv_t.
// (also copies the state before the step, alpha and breakdown included, to st_prev)
// q and z: float64, or float32 when qz_f32 (z rounded after r.z is formed).
hipError_t launch_cg_update(int ns, double* r, const void* q, void* z,
                            bool qz_f32, const double* minv, CgState* st, CgState* st_prev, int64_t n_obs,
                            int64_t vs, const double* minv_t, int64_t n_tail,
                            int n_rhs, const double* pq_part, int n_pq, double* partial_rz,
                            double* partial_rr, hipStream_t s);
// The scalar step (new rho, beta, residual, best iterate, convergence; st from
// st_prev and the update's partial sums; history[r * hist_stride + iter] = rel),
// then x += alpha p, x_best = x (RHS whose iterate became the best) and p = z + beta p
// (RHS that stepped); p32 (optional): also a float32 copy of the first n32 entries of
// each row of p (rows of stride vs32); p and z: float64, or float32 when p_f32 / z_f32
// (a float32 p, rows of stride nu, is the iteration's only direction: no p32 copy);
// x: float64, or with x_f32 (float32 p and z only) the float32 increment of the
// iterate since its last fold (launch_fold_f32), and then no best iterate is copied
hipError_t launch_cg_step_next(void* x, bool x_f32, double* xbest, void* p, bool p_f32, const void* z, bool z_f32,
                               CgState* st, const CgState* st_prev, const double* partial_rz,
                               const double* partial_rr, double* history, int hist_stride, int64_t nu, int n_rhs,
                               hipStream_t s, float* p32 = nullptr, int64_t n32 = 0, int64_t vs32 = 0);
hipError_t launch_apply_precond(int ns, const double* minv, const double* r, double* z,
                                int64_t n_obs, int64_t vs, const double* minv_t, int64_t n_tail,
                                int n_rhs, hipStream_t s);
hipError_t launch_axpby(double* y, const double* x, double a, double b, int64_t n, hipStream_t s);
hipError_t launch_sub(double* out, const double* a, const double* b, int64_t n, hipStream_t s);
// x[i] += d[i], then d[i] = 0, i < n (the float64 fold of a float32 increment)
hipError_t launch_fold_f32(double* x, float* d, int64_t n, hipStream_t s);

// ---------------------------------------------------------------- templates (k_template.hip)
// y[r][t] += p[r * vs + off + obs_idx[t]] where obs_idx[t] >= 0
hipError_t launch_onehot_gather(bool y_f64, const int32_t* obs_idx, const double* p, int64_t vs, int64_t off,
                                void* y, int64_t n_t, int n_rhs, hipStream_t s, const CgState* st = nullptr);
// y[r][t] += sum of the 32 HWP columns of t's segment times p[r * vs + off + 32 seg + i]
hipError_t launch_hwp_gather(bool y_f64, const SampleTile* tiles, int n_tiles, const int64_t* seg_start,
                             const float* omega, const double* p, int64_t vs, int64_t off, void* y, int64_t n_t,
                             int n_rhs, hipStream_t s, const CgState* st = nullptr);
// q[r * vs + off + 32 g + i] = sum over segment g of C[t][i] y[r][t] (tile partials in `partial`,
// [n_tiles][n_rhs][32]); with p also the block's p.q in pq_part[r * pq_stride + pq_slot]
hipError_t launch_hwp_scatter(bool y_f64, const SampleTile* tiles, int n_tiles, const int32_t* seg_tile, int n_seg,
                              const int64_t* seg_start, const float* omega, const void* y, int64_t n_t, int n_rhs,
                              double* partial, double* q, int64_t vs, int64_t off, const double* p,
                              double* pq_part, int pq_stride, int pq_slot, hipStream_t s,
                              const CgState* st = nullptr);
// diag[32 g + i] = sum over segment g of C[t][i]^2 w_t, w_t = f_b(0) (kind 0) or 1 (kind 1)
hipError_t launch_hwp_diag(int kind, const SampleTile* tiles, int n_tiles, const int32_t* seg_tile, int n_seg,
                           const int64_t* seg_start, const float* omega, const int64_t* iv_start, int n_iv,
                           const int32_t* iv_filter, const double* lags, int n_c, double* partial,
                           double* diag, hipStream_t s);
hipError_t launch_invert_diag(const double* d, double* out, int64_t n, hipStream_t s);
hipError_t launch_copy_rows(const double* src, int64_t src_stride, double* dst, int64_t dst_stride, int64_t n,
                            int n_rhs, hipStream_t s);
// y_out = f_b(0) y_in over tiles of the stationary intervals (white noise, n_c = 1)
hipError_t launch_white(bool out_f64, bool in_f64, const SampleTile* tiles, int n_tiles, const int32_t* iv_filter,
                        const double* lags, int n_c, const void* y_in, void* y_out, int64_t n_t, int n_rhs,
                        hipStream_t s, const CgState* st = nullptr);

}  // namespace mm
