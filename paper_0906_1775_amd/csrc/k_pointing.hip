// Pointing operators P (gather, map -> TOD) and P^T (scatter-add, TOD -> map).
//
// Formalism section of the MADmap paper: the row of sample t of P holds one
// unit weight for temperature, or (1/2, sin(2a_t)/2, cos(2a_t)/2) in the
// (I, Q, U) columns of its pixel for an ideal polarimeter; rows of excised
// samples are zero.
//
// Gather streams the time-ordered pointing (observed pixel id, sin/cos pair)
// coalesced and reads the map through the caches.  Scatter walks the
// pixel-major pointing built by the plan (as it is, a group of lanes per pixel,
// for pixels with many hits; else a sliced copy, one lane per pixel), so every
// pixel sum is formed in a fixed order and no atomics are needed.  The scatter can also return
// the per-block partial sums of p.q for the CG step length.  Maps are float64
// rows [R][vs] whose first n_obs * ns values are the observed pixels (the rest
// of a row holds template amplitudes).
#include <algorithm>

#include "mm_internal.h"

namespace mm {

// Each block covers kGatherUnroll x 256 consecutive samples; a thread takes
// samples tid, tid + 256, ... of its block, so every load and store instruction
// covers 64 consecutive samples of the wavefront.  A thread issues all its
// pointing loads, then all its map lookups, before any store: the lookups of
// one instruction then fall on the pixels of 64 consecutive samples, which a
// scan keeps within a few cache lines, and many independent chains are in
// flight per wavefront.  16 samples per thread (tiles of 4096): on 2^30 samples x 8
// RHS 1 % faster per iteration than 8, the same on one RHS; 4 and 32 are slower.
constexpr int kGatherUnroll = 16;

// one 8-byte nontemporal load of a (sin, cos) pair
__device__ __forceinline__ float2 load_nt(const float2* p) {
  const unsigned long long u = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(p));
  float2 r;
  __builtin_memcpy(&r, &u, sizeof(r));
  return r;
}

// The (I, Q, U) values of one pixel, read as one load
template <typename Tp> struct Stokes3 { Tp v[3]; };

// y_t = sum_s w_ts p_{pix_t, s} for the samples of row r; o must be a valid pixel:
// excised samples are clamped to pixel 0 by the caller and their value discarded,
// so that no lookup waits behind a branch.
template <int NS, typename Tp>
__device__ __forceinline__ double sky_value(const Tp* __restrict__ row, int32_t o, float s, float c) {
  if constexpr (NS == 1) {
    return (double)row[o];
  } else {
    const Stokes3<Tp> m = *reinterpret_cast<const Stokes3<Tp>*>(row + (int64_t)o * 3);
    return 0.5 * ((double)m.v[0] + (double)s * (double)m.v[1] + (double)c * (double)m.v[2]);
  }
}

// The samples t0 + u * 256 (u < kGatherUnroll) of one thread, t0 = its tile's first
// sample + threadIdx.x: y_t for every active RHS.
template <typename Ty, int NS, typename Tp>
__device__ __forceinline__ void gather_tile(const int32_t* __restrict__ pix_obs, const float2* __restrict__ w,
                                            const Tp* __restrict__ p, int64_t vs, Ty* __restrict__ y, int64_t n_t,
                                            int64_t ys, int n_rhs, const CgState* __restrict__ st, int64_t t0) {
  constexpr int U = kGatherUnroll;
  int32_t o[U];
  float2 sc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    // a slot past the last sample re-reads the last sample and is discarded;
    // the pointing streams are read once per pass: nontemporal, so they do not
    // evict the map (and the TOD rows other kernels re-read) from the caches
    const int64_t t = t0 + u * 256 < n_t ? t0 + u * 256 : n_t - 1;
    o[u] = __builtin_nontemporal_load(pix_obs + t);
    if (NS == 3) sc[u] = load_nt(w + t);
    else sc[u] = make_float2(0.f, 0.f);
  }
  for (int r = 0; r < n_rhs; ++r) {
    if (st && !st[r].active) continue;   // this RHS has stopped iterating
    const Tp* __restrict__ row = p + (int64_t)r * vs;
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double val = sky_value<NS, Tp>(row, o[u] >= 0 ? o[u] : 0, sc[u].x, sc[u].y);
      v[u] = o[u] >= 0 ? val : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t t = t0 + u * 256;
      if (t < n_t) y[(int64_t)r * ys + t] = (Ty)v[u];
    }
  }
}

// Tp: element type of the map (float64, or the float32 copy of the search
// direction that mixed-precision iterations gather from); y rows have stride ys.
// Requires n_obs >= 1 (pixel 0 exists).  Without `order` the blocks stride over
// the tiles in time order; with it block b takes one tile, the tiles sorted by
// the pixels they see: the hardware deals blocks to the 8 XCDs in turn, so block b
// takes sorted position (b mod 8) * ceil(n_tiles / 8) + b / 8, and the blocks an
// XCD runs at once read the map of one region of the sky through its L2.
template <typename Ty, int NS, typename Tp>
__global__ __launch_bounds__(256) void k_gather(const int32_t* __restrict__ pix_obs,
                                                const float2* __restrict__ w,
                                                const Tp* __restrict__ p, int64_t vs,
                                                Ty* __restrict__ y, int64_t n_t, int64_t ys, int n_rhs,
                                                const CgState* __restrict__ st,
                                                const int32_t* __restrict__ order, int64_t n_tiles) {
  constexpr int U = kGatherUnroll;
  if (st) {   // every RHS has stopped: nothing to read
    bool any = false;
    for (int r = 0; r < n_rhs; ++r) any = any || st[r].active != 0;
    if (!any) return;
  }
  if (order) {
    const int64_t per = (n_tiles + 7) / 8;
    const int64_t pos = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (pos >= n_tiles) return;
    gather_tile<Ty, NS, Tp>(pix_obs, w, p, vs, y, n_t, ys, n_rhs, st,
                            (int64_t)order[pos] * 256 * U + threadIdx.x);
    return;
  }
  const int64_t step = (int64_t)gridDim.x * 256 * U;
  for (int64_t t0 = (int64_t)blockIdx.x * 256 * U + threadIdx.x; t0 < n_t; t0 += step)
    gather_tile<Ty, NS, Tp>(pix_obs, w, p, vs, y, n_t, ys, n_rhs, st, t0);
}

hipError_t launch_gather(bool out_f64, int ns, const int32_t* pix_obs, const float* w,
                         const double* p, int64_t vs, void* y, int64_t n_t, int64_t n_obs, int n_rhs,
                         hipStream_t s, const CgState* st, const float* p32, int64_t vs32,
                         const int32_t* order) {
  if (n_t == 0) return hipSuccess;
  if (n_obs == 0)   // every sample excised: the TOD rows are zero (a fill kernel, safe under graph capture)
    return out_f64 ? launch_fill_f64((double*)y, 0.0, n_t * n_rhs, s)
                   : launch_fill_i32((int32_t*)y, 0, n_t * n_rhs, s);   // float32 zero = all bits zero
  const int64_t n_tiles = gather_tiles(n_t);
  int64_t nb = n_tiles;
  if (order) nb = 8 * ((n_tiles + 7) / 8);
  else if (nb > 65536) nb = 65536;
  const dim3 g((unsigned)nb), b(256);
  const float2* w2 = (const float2*)w;
#define MM_GA(TY, NS, TP, PP, VS) \
  hipLaunchKernelGGL((k_gather<TY, NS, TP>), g, b, 0, s, pix_obs, w2, PP, VS, (TY*)y, n_t, n_t, n_rhs, st, order, n_tiles)
  if (p32) {
    if (out_f64) { if (ns == 1) MM_GA(double, 1, float, p32, vs32); else MM_GA(double, 3, float, p32, vs32); }
    else { if (ns == 1) MM_GA(float, 1, float, p32, vs32); else MM_GA(float, 3, float, p32, vs32); }
  } else {
    if (out_f64) { if (ns == 1) MM_GA(double, 1, double, p, vs); else MM_GA(double, 3, double, p, vs); }
    else { if (ns == 1) MM_GA(float, 1, double, p, vs); else MM_GA(float, 3, double, p, vs); }
  }
#undef MM_GA
  return hipGetLastError();
}

int64_t gather_tiles(int64_t n_t) { return (n_t + 256 * kGatherUnroll - 1) / (256 * kGatherUnroll); }

// key[i] = the smallest observed id among the samples of gather tile i, -1 if it has none
__global__ __launch_bounds__(256) void k_tile_keys(const int32_t* __restrict__ pix_obs, int64_t n_t,
                                                   int32_t* __restrict__ key) {
  constexpr int64_t T = 256 * kGatherUnroll;
  const int64_t t0 = (int64_t)blockIdx.x * T;
  const int64_t t1 = t0 + T < n_t ? t0 + T : n_t;
  int32_t m = 0x7fffffff;
  for (int64_t t = t0 + threadIdx.x; t < t1; t += 256) {
    const int32_t o = pix_obs[t];
    if (o >= 0 && o < m) m = o;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int32_t v = __shfl_xor(m, off, 64);
    m = v < m ? v : m;
  }
  __shared__ int32_t wm[4];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t k = wm[0];
    for (int i = 1; i < 4; ++i) k = wm[i] < k ? wm[i] : k;
    key[blockIdx.x] = k == 0x7fffffff ? -1 : k;
  }
}

hipError_t launch_tile_keys(const int32_t* pix_obs, int64_t n_t, int32_t* key, hipStream_t s) {
  const int64_t n_tiles = gather_tiles(n_t);
  if (n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_keys, dim3((unsigned)n_tiles), dim3(256), 0, s, pix_obs, n_t, key);
  return hipGetLastError();
}

// dst[r * dst_stride + i] = (float)src[r * src_stride + i], i < n
__global__ void k_rows_to_f32(const double* __restrict__ src, int64_t ss, float* __restrict__ dst, int64_t ds,
                              int64_t n, int n_rhs) {
  const int64_t total = n * n_rhs;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += stride) {
    const int64_t r = k / n, i = k % n;
    dst[r * ds + i] = (float)src[r * ss + i];
  }
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

// Sliced layout of the pixel-major pointing: slice s holds the 64 observed
// pixels 64s .. 64s+63; entry (j, L) at sell_off[s] + 64 j + L is the j-th
// sample (in time order) of pixel 64s + L, or -1 past that pixel's hits.  A
// wavefront reads 64 consecutive entries per step, one per pixel, which for a
// raster scan are neighbouring TOD samples.
__global__ void k_sell_widths(const int64_t* __restrict__ pix_ptr, int64_t n_obs,
                              uint32_t* __restrict__ slice_len) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n_sl = (n_obs + 63) / 64;
  if (s >= n_sl) return;
  int64_t w = 0;
  for (int64_t o = s * 64; o < n_obs && o < s * 64 + 64; ++o) w = max(w, pix_ptr[o + 1] - pix_ptr[o]);
  slice_len[s] = (uint32_t)min(w * 64, (int64_t)0xFFFFFFFF);   // saturates; the host rejects it
}

// Fill of the sliced layout, a transpose of each slice's pixel-major runs: one
// workgroup per slice, whose wavefronts take interleaved tiles of kFillRows rows
// and stage each tile in LDS.  Reads take 16
// consecutive entries of 4 pixels per instruction (16 lanes per pixel); writes
// take a whole row (64 pixels) per instruction.  Rows are padded to kFillRows + 1
// entries so that both LDS access patterns are free of bank conflicts.
constexpr int kFillRows = 16;
constexpr int kFillWaves = 4;

__global__ __launch_bounds__(64 * kFillWaves) void k_sell_fill(
    const int64_t* __restrict__ pix_ptr, const int32_t* __restrict__ perm, const float2* __restrict__ w_pm,
    int64_t n_obs, const uint32_t* __restrict__ slice_end, const uint32_t* __restrict__ slice_len,
    int32_t* __restrict__ sell_t, float2* __restrict__ sell_w, int ns) {
  __shared__ int32_t s_t[kFillWaves][64][kFillRows + 1];
  __shared__ float2 s_w[kFillWaves][64][kFillRows + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int sub = lane / kFillRows, jj = lane % kFillRows;   // stage 1: pixel sub-index and row
  const int64_t n_sl = (n_obs + 63) / 64;
  for (int64_t s = blockIdx.x; s < n_sl; s += gridDim.x) {
    const int64_t base = (int64_t)slice_end[s] - slice_len[s];
    const int width = (int)(slice_len[s] / 64);
    const int64_t o = s * 64 + lane;
    const int64_t my_k0 = o < n_obs ? pix_ptr[o] : 0;
    const int my_cnt = o < n_obs ? (int)(pix_ptr[o + 1] - my_k0) : 0;
    for (int j0 = wv * kFillRows; j0 < width; j0 += kFillWaves * kFillRows) {   // uniform per wavefront
      // stage 1: pixel L = 4 q + sub, row j0 + jj; every load of the tile is issued
      // before the first LDS store (a slot past its pixel's hits re-reads the pixel's
      // first entry and is not stored), so they are all in flight together
      constexpr int NQ = 64 / (64 / kFillRows);
      int32_t tv[NQ];
      float2 wv2[NQ];
      bool in[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int L = q * (64 / kFillRows) + sub;
        const int64_t k0 = __shfl(my_k0, L, 64);
        const int cnt = __shfl(my_cnt, L, 64);
        const int j = j0 + jj;
        in[q] = j < cnt;
        const int64_t k = in[q] ? k0 + j : k0;
        tv[q] = cnt > 0 ? perm[k] : 0;
        if (ns == 3) wv2[q] = cnt > 0 ? w_pm[k] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int L = q * (64 / kFillRows) + sub;
        if (in[q]) {
          s_t[wv][L][jj] = tv[q];
          if (ns == 3) s_w[wv][L][jj] = wv2[q];
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      // stage 2: row j0 + r, pixel = lane
      const int rows = width - j0 < kFillRows ? width - j0 : kFillRows;
      for (int r = 0; r < rows; ++r) {
        const int64_t e = base + (int64_t)(j0 + r) * 64 + lane;
        const bool hit = j0 + r < my_cnt;
        sell_t[e] = hit ? s_t[wv][lane][r] : -1;
        if (ns == 3) sell_w[e] = hit ? s_w[wv][lane][r] : make_float2(0.f, 0.f);
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
  }
}

hipError_t launch_sell_widths(const int64_t* pix_ptr, int64_t n_obs, uint32_t* slice_len, hipStream_t s) {
  const int64_t n_sl = (n_obs + 63) / 64;
  if (n_sl == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sell_widths, dim3((unsigned)((n_sl + 255) / 256)), dim3(256), 0, s, pix_ptr, n_obs, slice_len);
  return hipGetLastError();
}

hipError_t launch_sell_fill(const int64_t* pix_ptr, const int32_t* perm, const float* w_pm, int64_t n_obs,
                            const uint32_t* slice_end, const uint32_t* slice_len, int32_t* sell_t,
                            float* sell_w, int ns, hipStream_t s) {
  const int64_t n_sl = (n_obs + 63) / 64;
  if (n_sl == 0) return hipSuccess;
  const int64_t nb = n_sl < 65536 ? n_sl : 65536;
  hipLaunchKernelGGL(k_sell_fill, dim3((unsigned)nb), dim3(64 * kFillWaves), 0, s, pix_ptr, perm,
                     (const float2*)w_pm, n_obs, slice_end, slice_len, sell_t, (float2*)sell_w, ns);
  return hipGetLastError();
}

// q = P^T y over the sliced layout.  WPS wavefronts share a slice: wavefront w
// adds the entries j = w, w + WPS, w + 2 WPS, ... of its lane's pixel,
// fetching kBatch entries ahead so that their loads overlap, and the WPS
// partial sums are combined in wavefront order through LDS.  Grid-stride over
// slices with a bounded grid (kScatterBlocks), so the optional p.q partial
// sums form a short, fixed list.
constexpr int kBlockWaves = 8;   // wavefronts per scatter block
constexpr int kBatch = 4;

// RG right-hand sides share one pass over the sliced pointing: the entries are
// loaded once per group and each RHS keeps its own accumulators, so the
// pointing is streamed ceil(R / RG) times instead of R times.  WPS wavefronts
// split a slice's entries (the plan picks 8 for pixels with hundreds of hits, 1
// for a few tens, where the cross-wave combine would dominate); a block of 8
// wavefronts works on 8 / WPS slices at a time.  Every (pixel, RHS) sum has a
// fixed order for a given WPS.  Tq: the element type q is stored in (the float64 sum is
// rounded to it); p (element type Tp, rows of stride ps) times the stored q gives the p.q
// partial sums.
template <typename Ty, typename Tq, typename Tp, int NS, int RG, int WPS>
__global__ __launch_bounds__(64 * kBlockWaves) void k_scatter(
    const uint32_t* __restrict__ slice_end, const uint32_t* __restrict__ slice_len,
    const int32_t* __restrict__ sell_t, const float2* __restrict__ sell_w, const Ty* __restrict__ y,
    Tq* __restrict__ q, int64_t vs, int64_t n_obs, int64_t n_t, int n_rhs, const Tp* __restrict__ p, int64_t ps,
    double* __restrict__ pq_part, int pq_stride, int pq_slot, const CgState* __restrict__ st) {
  constexpr int NW = kBlockWaves, SPB = NW / WPS;
  __shared__ double part[WPS > 1 ? NW : 1][RG * NS][64];
  __shared__ double sh[NW][RG];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int sg = wv / WPS, wi = wv % WPS;
  const int64_t n_sl = (n_obs + 63) / 64;
  for (int r0 = 0; r0 < n_rhs; r0 += RG) {
    bool act[RG];
    bool any = false;
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      act[g] = r0 + g < n_rhs && !(st && !st[r0 + g].active);   // RHS that stopped iterating are skipped
      any = any || act[g];
    }
    if (!any) continue;                    // uniform over the block
    double pq[RG];
#pragma unroll
    for (int g = 0; g < RG; ++g) pq[g] = 0.0;
    for (int64_t s0 = (int64_t)blockIdx.x * SPB; s0 < n_sl; s0 += (int64_t)gridDim.x * SPB) {
      const int64_t s = s0 + sg;
      const bool sv = s < n_sl;
      const int64_t base = sv ? (int64_t)slice_end[s] - slice_len[s] + lane : 0;
      const int width = sv ? (int)(slice_len[s] >> 6) : 0;
      Acc<Ty> a[RG][NS];
      for (int j0 = wi; j0 < width; j0 += WPS * kBatch) {
        // every load is issued unconditionally (a batch slot past the row re-reads the
        // row's last entry, a padding entry reads sample 0) and masked afterwards, so
        // that no load waits behind a branch
        int32_t tt[kBatch];
        float2 ww[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const int j = j0 + b * WPS;
          const int64_t e = base + (int64_t)(j < width ? j : width - 1) * 64;
          const int32_t tv = __builtin_nontemporal_load(sell_t + e);
          tt[b] = j < width ? tv : -1;
          if (NS == 3) ww[b] = load_nt(sell_w + e);
        }
#pragma unroll
        for (int g = 0; g < RG; ++g) {
          if (!act[g]) continue;
          const Ty* __restrict__ yr = y + (int64_t)(r0 + g) * n_t;
          Ty vv[kBatch];
#pragma unroll
          for (int b = 0; b < kBatch; ++b) {
            const Ty yv = yr[tt[b] >= 0 ? tt[b] : 0];
            vv[b] = tt[b] >= 0 ? yv : (Ty)0;
          }
#pragma unroll
          for (int b = 0; b < kBatch; ++b) {
            if (tt[b] < 0) continue;
            if (NS == 1) {
              a[g][0].add(vv[b]);
            } else {
              const Ty h = (Ty)0.5 * vv[b];
              a[g][0].add(h);
              a[g][1].add(h * (Ty)ww[b].x);
              a[g][2].add(h * (Ty)ww[b].y);
            }
          }
        }
      }
      const int64_t o = s * 64 + lane;
      if constexpr (WPS > 1) {
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
          for (int c = 0; c < NS; ++c) part[wv][g * NS + c][lane] = a[g][c].value();
        __syncthreads();
      }
      if (wi == 0 && sv && o < n_obs) {
#pragma unroll
        for (int g = 0; g < RG; ++g) {
          if (!act[g]) continue;
          const int64_t i = (int64_t)(r0 + g) * vs + o * NS;
          const int64_t ip = (int64_t)(r0 + g) * ps + o * NS;
#pragma unroll
          for (int c = 0; c < NS; ++c) {
            double v;
            if constexpr (WPS > 1) {
              v = part[sg * WPS][g * NS + c][lane];
#pragma unroll
              for (int w = 1; w < WPS; ++w) v += part[sg * WPS + w][g * NS + c][lane];
            } else {
              v = a[g][c].value();
            }
            const Tq vq = (Tq)v;
            q[i + c] = vq;
            if (p) pq[g] += (double)p[ip + c] * (double)vq;
          }
        }
      }
      if constexpr (WPS > 1) __syncthreads();
    }
    if (p) {   // block sums of the p.q contributions, fixed order
#pragma unroll
      for (int g = 0; g < RG; ++g) {
        double v = pq[g];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((tid & 63) == 0) sh[tid >> 6][g] = v;
      }
      __syncthreads();
      if (tid < RG && act[tid]) {
        double sum = 0.0;
        for (int w = 0; w < NW; ++w) sum += sh[w][tid];
        pq_part[(int64_t)(r0 + tid) * pq_stride + pq_slot + blockIdx.x] = sum;
      }
      __syncthreads();
    }
  }
}

// q = P^T y over the plain pixel-major layout: a wavefront takes 64 / kSegLanes
// neighbouring pixels at a time, kSegLanes lanes per pixel reading consecutive
// hits.  Those come from a few sweeps, which also hit the neighbours, so a TOD
// load touches fewer cache lines than the sliced layout's j-th hits of 64
// pixels (22.5 against 34.7 on a 2^24-sample raster).  For pixels with
// hundreds of hits, where the lanes stay busy, and a TOD the last-level cache
// mostly holds (neighbouring pixels' hits share TOD lines that this layout
// reads from different wavefronts).  Each lane sums its hits in order, then the
// lanes of a pixel are combined by a fixed butterfly in float64, so every
// (pixel, RHS) sum has a fixed order.
constexpr int kSegLanes = 16;
constexpr int kSegBatch = 4;   // loads in flight per lane
template <typename Ty, typename Tq, typename Tp, int NS, int RG>
__global__ __launch_bounds__(64 * kBlockWaves) void k_scatter_seg(
    const int64_t* __restrict__ pix_ptr, const int32_t* __restrict__ perm, const float2* __restrict__ w_pm,
    const Ty* __restrict__ y, Tq* __restrict__ q, int64_t vs, int64_t n_obs, int64_t n_t, int n_rhs,
    const Tp* __restrict__ p, int64_t ps, double* __restrict__ pq_part, int pq_stride, int pq_slot,
    const CgState* __restrict__ st) {
  constexpr int NW = kBlockWaves, G = kSegLanes, PPW = 64 / G;
  __shared__ double sh[NW][RG];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int gl = lane % G;   // lane within its pixel's group
  for (int r0 = 0; r0 < n_rhs; r0 += RG) {
    bool act[RG];
    bool any = false;
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      act[g] = r0 + g < n_rhs && !(st && !st[r0 + g].active);   // RHS that stopped iterating are skipped
      any = any || act[g];
    }
    if (!any) continue;                    // uniform over the block
    double pq[RG];
#pragma unroll
    for (int g = 0; g < RG; ++g) pq[g] = 0.0;
    for (int64_t o0 = ((int64_t)blockIdx.x * NW + wv) * PPW; o0 < n_obs; o0 += (int64_t)gridDim.x * NW * PPW) {
      const int64_t o = o0 + lane / G;
      const bool ov = o < n_obs;
      const int64_t k0 = ov ? pix_ptr[o] : 0, k1 = ov ? pix_ptr[o + 1] : 0;   // k1 > k0 for an observed pixel
      int span = (int)(k1 - k0);            // the wavefront walks its longest pixel
#pragma unroll
      for (int off = G; off < 64; off <<= 1) span = max(span, __shfl_xor(span, off, 64));
      Acc<Ty> a[RG][NS];
      for (int64_t j0 = 0; j0 < span; j0 += G * kSegBatch) {
        // loads issued unconditionally (a slot past the pixel's hits re-reads its
        // last one; a lane past the last pixel reads entry 0) and masked afterwards
        int32_t tt[kSegBatch];
        float2 ww[kSegBatch];
#pragma unroll
        for (int b = 0; b < kSegBatch; ++b) {
          const int64_t k = k0 + j0 + b * G + gl;
          const bool in = k < k1;
          const int64_t kk = in ? k : (k1 > 0 ? k1 - 1 : 0);
          const int32_t tv = __builtin_nontemporal_load(perm + kk);
          tt[b] = in ? tv : -1;
          if (NS == 3) ww[b] = load_nt(w_pm + kk);
        }
#pragma unroll
        for (int g = 0; g < RG; ++g) {
          if (!act[g]) continue;
          const Ty* __restrict__ yr = y + (int64_t)(r0 + g) * n_t;
          Ty vv[kSegBatch];
#pragma unroll
          for (int b = 0; b < kSegBatch; ++b) {
            const Ty yv = yr[tt[b] >= 0 ? tt[b] : 0];
            vv[b] = tt[b] >= 0 ? yv : (Ty)0;
          }
#pragma unroll
          for (int b = 0; b < kSegBatch; ++b) {
            if (tt[b] < 0) continue;
            if (NS == 1) {
              a[g][0].add(vv[b]);
            } else {
              const Ty h = (Ty)0.5 * vv[b];
              a[g][0].add(h);
              a[g][1].add(h * (Ty)ww[b].x);
              a[g][2].add(h * (Ty)ww[b].y);
            }
          }
        }
      }
#pragma unroll
      for (int g = 0; g < RG; ++g) {
        if (!act[g]) continue;
        const int64_t i = (int64_t)(r0 + g) * vs + o * NS;
        const int64_t ip = (int64_t)(r0 + g) * ps + o * NS;
#pragma unroll
        for (int c = 0; c < NS; ++c) {
          double v = a[g][c].value();
#pragma unroll
          for (int off = 1; off < G; off <<= 1) v += __shfl_xor(v, off, 64);   // same sum on the group's lanes
          const Tq vq = (Tq)v;
          if (ov && gl == c) q[i + c] = vq;
          if (p && ov && gl == 0) pq[g] += (double)p[ip + c] * (double)vq;
        }
      }
    }
    if (p) {   // block sums of the p.q contributions, fixed order
#pragma unroll
      for (int g = 0; g < RG; ++g) {
        double v = pq[g];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) sh[wv][g] = v;
      }
      __syncthreads();
      if (tid < RG && act[tid]) {
        double sum = 0.0;
        for (int w = 0; w < NW; ++w) sum += sh[w][tid];
        pq_part[(int64_t)(r0 + tid) * pq_stride + pq_slot + blockIdx.x] = sum;
      }
      __syncthreads();
    }
  }
}

int scatter_blocks(int64_t n_obs, int wps) {
  if (wps == 0) {
    const int64_t ppb = (int64_t)kBlockWaves * (64 / kSegLanes);   // pixels per block and step
    return (int)std::max<int64_t>(1, std::min<int64_t>((n_obs + ppb - 1) / ppb, kScatterBlocks));
  }
  const int64_t n_sl = (n_obs + 63) / 64;
  const int64_t spb = kBlockWaves / std::max(1, wps);
  return (int)std::max<int64_t>(1, std::min<int64_t>((n_sl + spb - 1) / spb, kScatterBlocks));
}

// wavefronts per slice for a layout whose pixels have `avg` entries on average
// (the plan may still choose 8 wavefronts per slice over 0 for a large TOD)
int scatter_waves_per_slice(double avg) { return avg >= 128 ? 0 : avg >= 64 ? 4 : avg >= 32 ? 2 : 1; }

template <typename Ty, typename Tq, typename Tp>
static hipError_t scatter_typed(int ns, const SellLayout& L, const Ty* y, Tq* q, int64_t vs, int64_t n_obs,
                                int64_t n_t, int n_rhs, hipStream_t s, const Tp* p, int64_t ps, double* pq_part,
                                int pq_stride, int pq_slot, const CgState* st) {
  if (n_obs == 0) return hipSuccess;
  const dim3 g((unsigned)scatter_blocks(n_obs, L.wps)), b(64 * kBlockWaves);
  if (L.wps == 0) {
    const float2* w = (const float2*)L.w_pm;
#define MM_SG(NS, RG) hipLaunchKernelGGL((k_scatter_seg<Ty, Tq, Tp, NS, RG>), g, b, 0, s, L.ptr, L.perm, w, y, q, \
                                         vs, n_obs, n_t, n_rhs, p, ps, pq_part, pq_stride, pq_slot, st)
    if (ns == 1) { if (n_rhs == 1) MM_SG(1, 1); else MM_SG(1, 4); }
    else { if (n_rhs == 1) MM_SG(3, 1); else MM_SG(3, 4); }
#undef MM_SG
    return hipGetLastError();
  }
  const float2* w = (const float2*)L.w;
#define MM_SC(NS, RG, WPS) hipLaunchKernelGGL((k_scatter<Ty, Tq, Tp, NS, RG, WPS>), g, b, 0, s, L.end, L.len, L.t, \
                                              w, y, q, vs, n_obs, n_t, n_rhs, p, ps, pq_part, pq_stride, pq_slot, st)
#define MM_SC_W(NS, RG)                        \
  switch (L.wps) {                             \
    case 1: MM_SC(NS, RG, 1); break;           \
    case 2: MM_SC(NS, RG, 2); break;           \
    case 4: MM_SC(NS, RG, 4); break;           \
    default: MM_SC(NS, RG, 8); break;          \
  }
  // one accumulator set for a single RHS; groups of 4 otherwise
  if (ns == 1) { if (n_rhs == 1) { MM_SC_W(1, 1) } else { MM_SC_W(1, 4) } }
  else { if (n_rhs == 1) { MM_SC_W(3, 1) } else { MM_SC_W(3, 4) } }
#undef MM_SC_W
#undef MM_SC
  return hipGetLastError();
}

hipError_t launch_scatter(bool in_f64, int ns, const SellLayout& L, const void* y, double* q, int64_t vs,
                          int64_t n_obs, int64_t n_t, int n_rhs, hipStream_t s, const double* p,
                          double* pq_part, int pq_stride, int pq_slot, const CgState* st) {
  if (in_f64)
    return scatter_typed<double, double, double>(ns, L, (const double*)y, q, vs, n_obs, n_t, n_rhs, s, p, vs,
                                                 pq_part, pq_stride, pq_slot, st);
  return scatter_typed<float, double, double>(ns, L, (const float*)y, q, vs, n_obs, n_t, n_rhs, s, p, vs, pq_part,
                                              pq_stride, pq_slot, st);
}

hipError_t launch_scatter_q32(int ns, const SellLayout& L, const float* y, float* q, int64_t vs, int64_t n_obs,
                              int64_t n_t, int n_rhs, hipStream_t s, const float* p32, int64_t vs32,
                              double* pq_part, int pq_stride, int pq_slot, const CgState* st) {
  return scatter_typed<float, float, float>(ns, L, y, q, vs, n_obs, n_t, n_rhs, s, p32, vs32, pq_part, pq_stride,
                                            pq_slot, st);
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

hipError_t launch_rows_to_f32(const double* src, int64_t src_stride, float* dst, int64_t dst_stride, int64_t n,
                              int n_rhs, hipStream_t s) {
  if (n == 0 || n_rhs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_to_f32, grid_for(n * n_rhs), dim3(256), 0, s, src, src_stride, dst, dst_stride, n, n_rhs);
  return hipGetLastError();
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

__global__ void k_to_observed(const double* __restrict__ glob, int64_t gs, double* __restrict__ obs, int64_t os,
                              const int32_t* __restrict__ obs2glob, int64_t n_obs, int ns, int n_rhs) {
  const int64_t per = n_obs * ns;
  const int64_t n = per * n_rhs;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int64_t r = i / per, rem = i % per, o = rem / ns, c = rem % ns;
    obs[r * os + rem] = glob[r * gs + (int64_t)obs2glob[o] * ns + c];
  }
}

// global map = observed values at observed pixels, 0 elsewhere (one pass over the global map)
__global__ void k_to_global(const double* __restrict__ obs, int64_t os, double* __restrict__ glob, int64_t gs,
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
      glob[r * gs + gp * ns + c] = seen ? obs[r * os + lo * ns + c] : 0.0;
  }
}

hipError_t launch_to_observed(const double* glob, int64_t glob_stride, double* obs, int64_t obs_stride,
                              const int32_t* obs2glob, int64_t n_obs, int64_t n_pix, int ns, int n_rhs,
                              hipStream_t s) {
  (void)n_pix;
  const int64_t n = n_obs * ns * n_rhs;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_observed, grid_for(n), dim3(256), 0, s, glob, glob_stride, obs, obs_stride, obs2glob,
                     n_obs, ns, n_rhs);
  return hipGetLastError();
}

hipError_t launch_to_global(const double* obs, int64_t obs_stride, double* glob, int64_t glob_stride,
                            const int32_t* obs2glob, int64_t n_obs, int64_t n_pix, int ns, int n_rhs,
                            hipStream_t s) {
  const int64_t n = n_pix * n_rhs;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_global, grid_for(n), dim3(256), 0, s, obs, obs_stride, glob, glob_stride, obs2glob,
                     n_obs, n_pix, ns, n_rhs);
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
