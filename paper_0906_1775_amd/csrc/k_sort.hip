// Plan-time pointing preparation: pixel range check, stable sort of samples
// by pixel, observed-pixel compaction and the pixel-major layout.
//
// The paper keeps three pixel index schemes (Implementation section, pixel
// indexing) and re-indexes with binary searches every time the pointing is
// rebuilt.  Here the pointing stays resident, so the re-indexing happens once:
// a stable least-significant-digit radix sort (8-bit digits, or 9-bit ones where
// they save a pass) orders the
// samples by pixel; the first sample of each run of equal pixels opens an
// observed pixel, which gives the observed ids, the pixel-major CSR offsets,
// hit counts and the time-major observed index used by the gather.
//
// Sort tile: 256 threads x 16 rounds = 4096 keys.  Within a round, lanes of a
// wavefront holding the same digit find each other with one ballot per digit bit; the
// per-wave counts in LDS order the four waves; rounds run in key order, so
// the sort is stable and every output position is computed, not raced for.
// Each tile is ordered by digit in LDS before it is written out.
#include "mm_internal.h"

namespace mm {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortThreads * kSortRounds;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanBlock = kScanThreads * kScanItems;

static dim3 grid_for(int64_t n, int threads = 256) {
  int64_t nb = (n + threads - 1) / threads;
  if (nb > 65536) nb = 65536;
  if (nb < 1) nb = 1;
  return dim3((unsigned)nb);
}

__global__ void k_check_pix(const int32_t* __restrict__ pix, int64_t n, int64_t n_pix,
                            int32_t* __restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t p = pix[i];
    bad |= (p < -1) || ((int64_t)p >= n_pix);
  }
  if (bad) flag[0] = 1;   // every writer stores the same value
}

hipError_t launch_check_pix(const int32_t* pix, int64_t n, int64_t n_pix, int32_t* flag,
                            hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_pix, grid_for(n), dim3(256), 0, s, pix, n, n_pix, flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------- scan (uint32)
// block scan of 4096 items; writes per-block totals
__global__ __launch_bounds__(kScanThreads) void k_scan_block(const uint32_t* __restrict__ in,
                                                             uint32_t* __restrict__ out, int64_t n,
                                                             uint32_t* __restrict__ block_sums,
                                                             int exclusive) {
  __shared__ uint32_t sh[kScanThreads];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)tid * kScanItems;
  uint32_t v[kScanItems];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    v[i] = idx < n ? in[idx] : 0u;
    sum += v[i];
  }
  sh[tid] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan of the 256 thread sums
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint32_t x = tid >= off ? sh[tid - off] : 0u;
    __syncthreads();
    sh[tid] += x;
    __syncthreads();
  }
  uint32_t run = tid > 0 ? sh[tid - 1] : 0u;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    const uint32_t x = v[i];
    if (exclusive) {
      if (idx < n) out[idx] = run;
      run += x;
    } else {
      run += x;
      if (idx < n) out[idx] = run;
    }
  }
  if (tid == kScanThreads - 1) block_sums[blockIdx.x] = sh[kScanThreads - 1];
}

__global__ void k_scan_add(uint32_t* __restrict__ out, int64_t n,
                           const uint32_t* __restrict__ block_offsets) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += block_offsets[i / kScanBlock];
}

size_t scan_scratch_bytes(int64_t n) {
  size_t total = 0;
  int64_t m = n;
  while (m > 1) {
    const int64_t nb = (m + kScanBlock - 1) / kScanBlock;
    total += (size_t)(nb + 1) * sizeof(uint32_t);
    if (nb == 1) break;
    m = nb;
  }
  return total + 64;
}

static hipError_t scan_impl(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* scratch,
                            int exclusive, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  uint32_t* sums = scratch;
  hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n, sums,
                     exclusive);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nb == 1) return e;
  // exclusive scan of the block totals, in place, then add
  e = scan_impl(sums, sums, nb, scratch + nb + 1, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, sums);
  return hipGetLastError();
}

hipError_t launch_scan_inclusive(const uint32_t* in, uint32_t* out, int64_t n, void* scratch,
                                 hipStream_t s) {
  return scan_impl(in, out, n, (uint32_t*)scratch, 0, s);
}

// ---------------------------------------------------------------- observed ids
// seg[i] = number of runs of equal valid keys (key < n_pix) that start at or
// before i, for the sorted keys: the run-start flags are formed on the fly and
// scanned block by block (4096 items); the sample after the last valid key
// writes n_valid.  Keys go through LDS so that global loads and stores stay
// coalesced while each thread scans 16 consecutive items; LDS slots are padded
// by one word per 16 so that the per-thread runs spread over the banks.
__device__ __forceinline__ int seg_pad(int j) { return j + (j >> 4); }

__global__ __launch_bounds__(kScanThreads) void k_seg_scan_block(const uint32_t* __restrict__ keys, int64_t n,
                                                                 uint32_t n_pix, uint32_t* __restrict__ out,
                                                                 uint32_t* __restrict__ block_sums,
                                                                 int64_t* __restrict__ n_valid) {
  __shared__ uint32_t sk[kScanBlock + kScanBlock / 16 + 2];   // padded keys b0 .. b0 + 4095
  __shared__ uint32_t sh[kScanThreads];
  __shared__ uint32_t edge[2];                                 // keys b0 - 1 and b0 + 4096
  const int tid = threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int j = i * kScanThreads + tid;
    const int64_t idx = b0 + j;
    sk[seg_pad(j)] = idx < n ? keys[idx] : 0xFFFFFFFFu;
  }
  if (tid == 0) {
    edge[0] = b0 > 0 ? keys[b0 - 1] : 0xFFFFFFFFu;
    edge[1] = b0 + kScanBlock < n ? keys[b0 + kScanBlock] : 0xFFFFFFFFu;
  }
  __syncthreads();
  uint32_t v[kScanItems];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int j = tid * kScanItems + i;
    const int64_t idx = b0 + j;
    const uint32_t k = sk[seg_pad(j)];
    const uint32_t prev = j > 0 ? sk[seg_pad(j - 1)] : edge[0];
    const uint32_t next = j + 1 < kScanBlock ? sk[seg_pad(j + 1)] : edge[1];
    const bool valid = idx < n && k < n_pix;
    v[i] = (valid && (idx == 0 || prev != k)) ? 1u : 0u;
    sum += v[i];
    if (valid && (idx == n - 1 || next >= n_pix)) n_valid[0] = idx + 1;   // unique writer
  }
  sh[tid] = sum;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint32_t x = tid >= off ? sh[tid - off] : 0u;
    __syncthreads();
    sh[tid] += x;
    __syncthreads();
  }
  uint32_t run = tid > 0 ? sh[tid - 1] : 0u;
  if (tid == kScanThreads - 1) block_sums[blockIdx.x] = sh[kScanThreads - 1];
  // inclusive values back through LDS, then coalesced stores
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    run += v[i];
    sk[seg_pad(tid * kScanItems + i)] = run;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int j = i * kScanThreads + tid;
    const int64_t idx = b0 + j;
    if (idx < n) out[idx] = sk[seg_pad(j)];
  }
}

hipError_t launch_segment_scan(const uint32_t* keys, int64_t n, uint32_t n_pix, uint32_t* seg, int64_t* n_valid,
                               void* scratch, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  uint32_t* sums = (uint32_t*)scratch;
  hipLaunchKernelGGL(k_seg_scan_block, dim3((unsigned)nb), dim3(kScanThreads), 0, s, keys, n, n_pix, seg, sums,
                     n_valid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nb == 1) return e;
  e = scan_impl(sums, sums, nb, sums + nb + 1, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seg, n, sums);
  return hipGetLastError();
}

// ---------------------------------------------------------------- radix sort
__global__ void k_sort_init(const int32_t* __restrict__ pix, int64_t n, uint32_t n_pix,
                            uint32_t* __restrict__ keys, int32_t* __restrict__ vals) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t p = pix[i];
    keys[i] = p >= 0 ? (uint32_t)p : n_pix;
    vals[i] = (int32_t)i;
  }
}

// Digit counts of one tile (digits of BITS bits at `shift`), digit-major:
// counts[d * n_tiles + tile].
template <int BITS>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                             int64_t n, int shift, int64_t n_tiles,
                                                             uint32_t* __restrict__ counts) {
  constexpr int NB = 1 << BITS, PER = NB / kSortThreads;
  __shared__ uint32_t h[NB];
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < PER; ++q) h[q * kSortThreads + tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
  for (int i = 0; i < kSortRounds; ++i) {
    const int64_t idx = base + (int64_t)i * kSortThreads + tid;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & (NB - 1)], 1u);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q)
    counts[(int64_t)(q * kSortThreads + tid) * n_tiles + blockIdx.x] = h[q * kSortThreads + tid];
}

// Stable scatter of one tile by digit.  Each wavefront ranks its own quarter
// of the tile (keys in tile order, 64 per round) against running per-digit
// counts that only it touches, so the rounds need no block barrier: lanes with
// the same digit find each other with BITS ballots.  The per-wave counts then
// give each wave its offset within every digit, the tile is placed in LDS in
// (digit, rank) order and written out in that order, so each digit's keys
// leave as one contiguous run at offsets[digit][tile] instead of one scattered
// word per key.
template <int BITS>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t* __restrict__ keys_in, const int32_t* __restrict__ vals_in, int64_t n, int shift,
    int64_t n_tiles, const uint32_t* __restrict__ offsets, uint32_t* __restrict__ keys_out,
    int32_t* __restrict__ vals_out) {
  constexpr int NB = 1 << BITS, PER = NB / kSortThreads;   // digits per thread in the per-digit loops
  constexpr int NW = kSortThreads / 64, KPW = kSortTile / NW;   // wavefronts, keys per wavefront
  __shared__ uint32_t s_key[kSortTile];
  __shared__ int32_t s_val[kSortTile];
  __shared__ uint32_t gbase[NB];                    // output offset of this tile's digit d
  __shared__ uint32_t lstart[NB];                   // first LDS slot of digit d
  __shared__ uint32_t wcnt[NW][NB];                 // keys of digit d in wave w's quarter, then the
                                                    // keys of digit d in the quarters before it
  __shared__ uint32_t tsum[NW];                     // wave totals of the digit scan
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int d = q * kSortThreads + tid;
    gbase[d] = offsets[(int64_t)d * n_tiles + blockIdx.x];
#pragma unroll
    for (int w = 0; w < NW; ++w) wcnt[w][d] = 0;
  }
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
  const int n_here = (int)((n - tile0) < kSortTile ? (n - tile0) : kSortTile);
  uint32_t key[kSortRounds], rk[kSortRounds];
  int32_t val[kSortRounds];
#pragma unroll
  for (int i = 0; i < kSortRounds; ++i) {
    const int j = wave * KPW + i * 64 + lane;
    const bool valid = j < n_here;
    key[i] = valid ? keys_in[tile0 + j] : 0u;
    val[i] = valid ? vals_in[tile0 + j] : 0;
  }
#pragma unroll
  for (int i = 0; i < kSortRounds; ++i) {
    const int j = wave * KPW + i * 64 + lane;
    const bool valid = j < n_here;
    const uint32_t d = (key[i] >> shift) & (NB - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
    const uint32_t before = wcnt[wave][d];
    rk[i] = before + rank;
    // every lane has read its count before the digit's first lane writes the new one
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) wcnt[wave][d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();
  // per digit: the waves' counts become offsets within the digit; exclusive scan of
  // the tile's NB digit totals: thread tid owns the PER consecutive digits tid * PER ..;
  // a scan of the 256 thread sums (within each wavefront, then across the four) orders them
  {
    uint32_t c[PER], tot = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int d = tid * PER + q;
      uint32_t run = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const uint32_t x = wcnt[w][d];
        wcnt[w][d] = run;
        run += x;
      }
      c[q] = run;
      tot += run;
    }
    // inclusive scan of the thread sums within the wavefront, then the wave totals
    uint32_t incl = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(incl, off, 64);
      if (lane >= off) incl += y;
    }
    if (lane == 63) tsum[wave] = incl;
    __syncthreads();
    uint32_t run = incl - tot;
    for (int w = 0; w < wave; ++w) run += tsum[w];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      lstart[tid * PER + q] = run;
      run += c[q];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kSortRounds; ++i) {
    const int j = wave * KPW + i * 64 + lane;
    if (j < n_here) {
      const uint32_t d = (key[i] >> shift) & (NB - 1);
      const uint32_t pos = lstart[d] + wcnt[wave][d] + rk[i];
      s_key[pos] = key[i];
      s_val[pos] = val[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kSortRounds; ++i) {
    const int j = i * kSortThreads + tid;
    if (j < n_here) {
      const uint32_t k = s_key[j];
      const uint32_t d = (k >> shift) & (NB - 1);
      const uint32_t pos = gbase[d] + ((uint32_t)j - lstart[d]);
      keys_out[pos] = k;
      vals_out[pos] = s_val[j];
    }
  }
}

// widest digit of a pass (9-bit digits are used where they save a pass)
constexpr int kSortMaxBits = 9;

size_t sort_scratch_bytes(int64_t n) {
  const int64_t n_tiles = (n + kSortTile - 1) / kSortTile;
  const int64_t m = (int64_t(1) << kSortMaxBits) * n_tiles;
  return (size_t)n * 8 * 2                      // two key/value buffers
         + (size_t)m * sizeof(uint32_t)          // digit counts / offsets
         + scan_scratch_bytes(m) + 256;
}

hipError_t launch_sort_by_pixel(const int32_t* pix, int64_t n, int64_t n_pix, uint32_t* keys_out,
                                int32_t* vals_out, void* scratch, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t n_tiles = (n + kSortTile - 1) / kSortTile;
  char* p = (char*)scratch;
  uint32_t* ka = (uint32_t*)p; p += (size_t)n * 4;
  int32_t* va = (int32_t*)p;   p += (size_t)n * 4;
  uint32_t* kb = (uint32_t*)p; p += (size_t)n * 4;
  int32_t* vb = (int32_t*)p;   p += (size_t)n * 4;
  uint32_t* counts = (uint32_t*)p; p += (size_t)((int64_t(1) << kSortMaxBits) * n_tiles) * 4;
  uint32_t* scan_tmp = (uint32_t*)p;

  int bits = 0;
  while (bits < 32 && (((uint64_t)n_pix) >> bits) != 0) ++bits;   // keys lie in [0, n_pix]
  // 8-bit digits, or 9-bit ones where they save a pass of up to three (keys of 9, 17 or
  // 18 bits: the pass they save sorts one or two bits).  A tile of 4,096 keys spread
  // over 512 digits leaves in runs of 8 keys, half the write runs of 256 digits, so
  // for wider keys (a 2^30-sample, 26-bit sort: 3 x 9 bits took 104 ms against 96 ms
  // for 4 x 8) the fourth 8-bit pass is the cheaper choice.
  int passes = (bits + 7) / 8;
  if (passes == 0) passes = 1;
  const int dbits = (passes > 1 && passes <= 3 && (passes - 1) * kSortMaxBits >= bits) ? kSortMaxBits : 8;
  if (dbits == kSortMaxBits) passes -= 1;

  hipLaunchKernelGGL(k_sort_init, grid_for(n), dim3(256), 0, s, pix, n, (uint32_t)n_pix, ka, va);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint32_t *kin = ka, *kout = kb;
  int32_t *vin = va, *vout = vb;
  for (int ps = 0; ps < passes; ++ps) {
    const int shift = dbits * ps;
    const bool last = ps == passes - 1;
    uint32_t* ko = last ? keys_out : kout;
    int32_t* vo = last ? vals_out : vout;
    const int64_t m = (int64_t(1) << dbits) * n_tiles;
    if (dbits == 8)
      hipLaunchKernelGGL(k_radix_hist<8>, dim3((unsigned)n_tiles), dim3(kSortThreads), 0, s, kin, n, shift, n_tiles,
                         counts);
    else
      hipLaunchKernelGGL(k_radix_hist<kSortMaxBits>, dim3((unsigned)n_tiles), dim3(kSortThreads), 0, s, kin, n, shift,
                         n_tiles, counts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_impl(counts, counts, m, scan_tmp, 1, s)) != hipSuccess) return e;
    if (dbits == 8)
      hipLaunchKernelGGL(k_radix_scatter<8>, dim3((unsigned)n_tiles), dim3(kSortThreads), 0, s, kin, vin, n, shift,
                         n_tiles, counts, ko, vo);
    else
      hipLaunchKernelGGL(k_radix_scatter<kSortMaxBits>, dim3((unsigned)n_tiles), dim3(kSortThreads), 0, s, kin, vin, n,
                         shift, n_tiles, counts, ko, vo);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    uint32_t* tk = kin; kin = kout; kout = tk;
    int32_t* tv = vin; vin = vout; vout = tv;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------- observed layout
// seg_id = observed id + 1 of each sorted valid sample (launch_segment_scan)
__global__ void k_build_layout(const uint32_t* __restrict__ keys, const int32_t* __restrict__ vals,
                               const uint32_t* __restrict__ seg_id, int64_t n, uint32_t n_pix,
                               const float2* __restrict__ w, int ns, int64_t* __restrict__ pix_ptr,
                               int32_t* __restrict__ obs2glob, float2* __restrict__ w_pm,
                               int32_t* __restrict__ perm) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t k = keys[i];
    const int32_t v = vals[i];
    if (k < n_pix) {
      const int32_t o = (int32_t)seg_id[i] - 1;
      if (i == 0 || keys[i - 1] != k) {
        pix_ptr[o] = i;
        obs2glob[o] = (int32_t)k;
      }
      perm[i] = v;
      if (ns == 3) w_pm[i] = w[v];
    }
  }
}

// glob2obs[obs2glob[o]] = o (the entries of unobserved pixels are set to -1 beforehand)
__global__ void k_invert_obs(const int32_t* __restrict__ obs2glob, int64_t n_obs, int32_t* __restrict__ glob2obs) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n_obs; o += stride)
    glob2obs[obs2glob[o]] = (int32_t)o;
}

// time-major observed index: pix_obs[t] = glob2obs[key[t]], -1 for excised samples
__global__ void k_obs_index(const int32_t* __restrict__ key, int64_t n, const int32_t* __restrict__ glob2obs,
                            int32_t* __restrict__ pix_obs) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
    const int32_t k = key[t];
    pix_obs[t] = k >= 0 ? glob2obs[k] : -1;
  }
}

hipError_t launch_obs_index(const int32_t* key, int64_t n, const int32_t* obs2glob, int64_t n_obs,
                            int32_t* glob2obs, int64_t n_keys, int32_t* pix_obs, hipStream_t s) {
  hipError_t e = launch_fill_i32(glob2obs, -1, n_keys, s);
  if (e != hipSuccess) return e;
  if (n_obs > 0) {
    hipLaunchKernelGGL(k_invert_obs, grid_for(n_obs), dim3(256), 0, s, obs2glob, n_obs, glob2obs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_obs_index, grid_for(n), dim3(256), 0, s, key, n, glob2obs, pix_obs);
  return hipGetLastError();
}

hipError_t launch_build_layout(const uint32_t* keys, const int32_t* vals, const uint32_t* seg_id,
                               int64_t n, uint32_t n_pix, const float* w, int ns, int64_t* pix_ptr,
                               int32_t* obs2glob, float* w_pm, int32_t* perm, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_layout, grid_for(n), dim3(256), 0, s, keys, vals, seg_id, n, n_pix,
                     (const float2*)w, ns, pix_ptr, obs2glob, (float2*)w_pm, perm);
  return hipGetLastError();
}

}  // namespace mm
