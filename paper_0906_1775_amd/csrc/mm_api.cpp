// C ABI of the map-maker: plan construction, operator entry points and the
// PCG driver.  See include/mm.h for the contract of every entry point.
#include "mm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mm_internal.h"

using namespace mm;

namespace {

thread_local std::string g_last_error;

struct Failure {
  mm_status_t status;
};

[[noreturn]] void fail(mm_status_t st, const std::string& msg) {
  g_last_error = msg;
  throw Failure{st};
}

void hipchk(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      fail(MM_ENOMEM, std::string(what) + ": " + hipGetErrorString(e));
    fail(MM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}

template <typename F>
mm_status_t guarded(F&& f) {
  try {
    g_last_error.clear();
    f();
    return MM_OK;
  } catch (const Failure& x) {
    return x.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return MM_ENOMEM;
  } catch (...) {
    g_last_error = "unexpected exception";
    return MM_EDEVICE;
  }
}

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
// Mixed solver: a check replaces the residual of an RHS whose recurrence residual fell
// below kMixedReplaceFall x its float64 residual at the last replacement, and blocks
// are sized so that it is not predicted to fall more than kMixedMaxDrop decades below
// that residual before the next check.
constexpr double kMixedReplaceFall = 1e-3;
constexpr double kMixedMaxDrop = 4.5;
constexpr int kMixedFirstBlock = 8;
// float64 residual below which (for every RHS) the float32 iteration moves x by a
// float32 increment: earlier increments are large enough that their rounding stays
// visible in the map (2^30-sample workload, increments from the first replacement
// on: map error at tol 1e-8 up by 4e-4 relative, one more tolerance step to reach
// the float64 solve's map error)
constexpr double kIncrementFrom = 1e-5;

// pinned staging slots of a plan (8 bytes each) and its dot-partial buffer
constexpr int kPinSlots = 8;
enum PinSlot { kPinFlag = 0, kPinObs, kPinValid, kPinTotal, kPinSingular };

int ilog2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

// transform length the plan prefers when the descriptor leaves n_f open
constexpr int kPreferredMaxLogN = 13;   // n_f = 2^14
constexpr int kMinLogN = 6;

int32_t fft_length_rule(int32_t n_c, int64_t longest) {
  if (n_c < 1 || longest < 1) return 0;
  auto hprime_sign = [&](double nf) { return nf - 2.0 * n_c * (1.0 + std::log(nf)); };
  int64_t nf = 1;
  while (nf < longest) nf <<= 1;
  if (nf <= 2 * (int64_t)n_c) {
    nf = 1;
    while (nf <= 2 * (int64_t)n_c) nf <<= 1;
  } else if (hprime_sign((double)nf) > 0) {
    for (;;) {
      const int64_t half = nf / 2;
      if (half <= 2 * (int64_t)n_c || hprime_sign((double)half) < 0) break;
      nf = half;
    }
  }
  return nf > (int64_t(1) << 30) ? 0 : (int32_t)nf;
}

struct FilterSetup {
  bool ready = false;
  bool fp64 = true;
  int logn = 0;
  int variant = 0;         // workgroup shape of the transform (ols_variant_exists)
  int N = 0, nf = 0, m = 0;
  void* tw2 = nullptr;     // exp(-2 pi i k / n_f), k < N (real-to-complex packing)
  void* ptw = nullptr;     // per-pass twiddle tables of the transform (long: of its 2^8-point columns)
  void* spec = nullptr;
  bool long_path = false;  // n_f beyond one workgroup: the batched four-step transform (launch_ols_long)
  void* ptw_b = nullptr;   // long: per-pass twiddle tables of its rows
  void* ltab = nullptr;    // long: W_N and pairing twiddle tables (launch_long_tables)
  void* work = nullptr;    // long: intermediates of `batch` jobs
  int64_t batch = 0;
  OlsChunk* chunks = nullptr;
  std::vector<OlsChunk> chunks_host;   // source of the asynchronous upload of chunks, kept with the setup
  int n_chunks = 0;
};

// Streams of destroyed plans, kept per device for later plans of the process
// (creating a stream costs more than the small plans' kernels).
struct StreamPool {
  std::mutex mu;
  std::vector<hipStream_t> streams[64];
};

StreamPool& stream_pool() {
  static StreamPool* c = new StreamPool();   // never destroyed: streams outlive static teardown
  return *c;
}

hipStream_t stream_take(int dev) {
  if (dev >= 0 && dev < 64) {
    StreamPool& c = stream_pool();
    std::lock_guard<std::mutex> lk(c.mu);
    if (!c.streams[dev].empty()) {
      hipStream_t st = c.streams[dev].back();
      c.streams[dev].pop_back();
      return st;
    }
  }
  hipStream_t st = nullptr;
  hipchk(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "stream");
  return st;
}

void stream_put(int dev, hipStream_t st) {
  if (dev >= 0 && dev < 64) {
    StreamPool& c = stream_pool();
    std::lock_guard<std::mutex> lk(c.mu);
    if (c.streams[dev].size() < 16) {
      c.streams[dev].push_back(st);
      return;
    }
  }
  (void)hipStreamDestroy(st);
}

// Device memory of a plan: one block, the caller's workspace (mm_plan) or one the
// library allocated (mm_plan_create), cut into two regions.  Persistent data
// (pointing layouts, filters, preconditioner, scalars) are bumped from the start,
// up to a limit the descriptor bounds; the work region after it holds the TOD and
// CG work vectors.  Temporaries are stacked over the work region: during the build
// from its start (the work vectors are not in use before the build has finished,
// and every entry point waits for it), afterwards above the two TOD work buffers.
constexpr size_t kAlign = 256;
inline size_t align_up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }
inline size_t block_bytes(int64_t count, size_t elem) { return align_up((size_t)std::max<int64_t>(count, 1) * elem); }

// Entries of the device history ring of every RHS: the host copies it after each
// block of iterations, and blocks are shorter than the ring.
constexpr int kHistRing = 1024;
constexpr int kMaxCheckEvery = 256;   // blocks are at most 2 x check_every iterations

// Pixel-major layout of one pointing matrix with one non-zero per row: the sky
// pointing, or a one-hot template read as a temperature-only pointing.
struct Layout {
  int64_t n_obs = 0, n_valid = 0;
  int32_t* obs_idx = nullptr;    // [n_t] observed id of each sample, -1 = none (time-major)
  int64_t* ptr = nullptr;        // [n_obs + 1] CSR offsets of the pixel-major order
  int32_t* obs2glob = nullptr;   // [n_obs] global id of each observed id (sorted)
  int32_t* perm = nullptr;       // [n_valid] sample ids, pixel-major (released once sliced)
  float* w_pm = nullptr;         // [n_valid][2] (sin, cos), pixel-major (released once sliced)
  int group = 8;                 // lanes per pixel in the plan-time preconditioner build
  int wps = 0;                   // wavefronts per slice of the scatter (0: pixel-major arrays as they are)
  SellLayout sell;               // sliced pointing of the scatter
  int64_t sell_entries = 0;
};

// One block of template columns appended to the pointing.
struct Template {
  int kind = 0;
  int64_t n_glob = 0;            // amplitudes in map-shaped API buffers
  int64_t n_unk = 0;             // unknowns in the iteration vectors
  int64_t goff = 0;              // offset of its amplitudes after the map values (API layout)
  int64_t ooff = 0;              // offset after the map values (iteration layout)
  int pq_slot = 0, pq_n = 0;     // its p.q partial sums
  Layout lay;                    // one-hot: the index as a pointing
  const float* omega = nullptr;  // HWP: polarizer angle per sample
  int n_seg = 0;
  std::vector<int64_t> seg_host;
  int64_t* d_seg = nullptr;      // [n_seg + 1]
  int32_t* d_seg_tile = nullptr; // [n_seg + 1] first tile of each segment
  SampleTile* tiles = nullptr;
  int n_tiles = 0;
  double* partial = nullptr;     // [n_tiles][R][32] tile partial sums of the scatter
};

}  // namespace

struct mm_plan_s {
  // descriptor
  int ns = 1;
  int64_t n_pix = 0, n_t = 0;
  int n_iv = 0, n_filt = 0, n_c = 0;
  int precision = MM_FP64, precond = MM_PRECOND_BLOCK, R = 1;
  int nf_req = 0;
  int shape_req = 0;            // requested transform shape (0 = default)
  int solves = 0;               // solves completed with this plan
  int64_t lag_len = 0;
  double f_samp = 0;
  std::vector<int64_t> iv_start;
  std::vector<int32_t> iv_filter;
  std::vector<double> params;
  int device = 0;
  hipStream_t own = nullptr;    // stream of mm_solve and its graphs
  hipEvent_t ev_in = nullptr, ev_out = nullptr;

  // pointing
  int64_t n_obs = 0, n_valid = 0;
  const float* w = nullptr;     // caller's (sin, cos) pairs, time-major
  Layout px;                    // sky pointing
  int32_t* gather_order = nullptr;   // gather tiles sorted by the pixels they see, or null (time order)

  // templates
  std::vector<Template> tmpl;
  int64_t n_tglob = 0, n_tunk = 0;   // template amplitudes (API layout / iteration layout)
  double* minv_t = nullptr;          // [n_tunk] diagonal preconditioner of the amplitudes
  int n_pq = 0;                      // p.q partial sums per RHS over all scatters
  SampleTile* white_tiles = nullptr; // n_c = 1: tiles of the stationary intervals
  int n_white_tiles = 0;

  // noise
  double* lags = nullptr;
  double* d_params = nullptr;    // [n_filters][3] (sigma, f_knee, alpha) when given
  int64_t* d_iv_start = nullptr;
  int32_t* d_iv_hint = nullptr;   // coarse index of the interval table (build_interval_hint)
  std::vector<int32_t> iv_hint;   // its host copy, the source of the asynchronous upload
  int iv_hint_shift = 0;
  int32_t* d_iv_filter = nullptr;
  FilterSetup fs_main, fs64;

  // preconditioner
  double* minv = nullptr;
  int n_singular = 0;
  hipEvent_t ev_singular = nullptr;   // recorded after n_singular's copy to its pinned slot (null once read)

  // work
  void* y1 = nullptr;            // [R][n_t] of the iteration precision
  void* y2 = nullptr;
  double* y64a = nullptr;        // [n_t] float64 views of y1 / y2 (true residual in mixed mode)
  double* y64b = nullptr;
  double *vx = nullptr, *vp = nullptr, *vr = nullptr, *vz = nullptr, *vq = nullptr,
         *vxb = nullptr, *vb = nullptr;   // [R][nu]
  double *part1 = nullptr, *part2 = nullptr, *part3 = nullptr;
  double* part_pq = nullptr;     // [R][n_pq] partial sums of p.q
  float* vp32 = nullptr;         // [R][n_obs * ns] float32 copy of p's map part (mixed plans)
  double *vb64 = nullptr, *vxbest = nullptr;   // mixed refinement: b and the best iterate in float64
  double* vxacc = nullptr;                      // accumulated map of the restarted correction
  // set while a reliable-update solve runs float32 iterations: x then moves by a float32
  // increment held in the first half of vxb (which that solve does not otherwise use),
  // folded into the float64 vx for the RHS of each residual replacement
  bool x_inc32 = false;
  float* vdx32() const { return reinterpret_cast<float*>(vxb); }
  CgState* st = nullptr;
  CgState* st_prev = nullptr;    // state before the current step (written by the update)
  CgState* st_host = nullptr;     // pinned: the CG states, then the staging slots below
  char* pin = nullptr;            // pinned staging of scalar readbacks (kPinSlots 8-byte slots) and dot partials
  template <typename T>
  T* slot(int k) { return reinterpret_cast<T*>(pin + 8 * k); }
  double* pin_dots() { return reinterpret_cast<double*>(pin + kPinSlots * 8); }
  double* hist = nullptr;         // [R][kHistRing] residual per iteration (ring, index iter % kHistRing)
  double* hist_host = nullptr;    // pinned copy target of hist

  // cached graphs of check_every iterations, one per x mode (index x_inc32)
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  int graph_k[2] = {0, 0};

  hipEvent_t ev_ready = nullptr;  // recorded on the build stream when the plan's build work is queued

  // ---- device memory (see align_up): ws[0, pers_lim) persistent, ws[pers_lim, ws_size) work region
  char* ws = nullptr;
  size_t ws_size = 0;
  bool ws_owned = false;          // allocated by mm_plan_create (freed by mm_destroy)
  size_t pers_lim = 0, pers_top = 0;
  size_t work_top = 0;            // work vectors, bumped from pers_lim
  size_t tmp_base = 0;            // temporaries are stacked from here
  size_t tmp_peak = 0;            // highest end of a temporary so far
  struct Tmp {
    size_t off, bytes;
    bool live;
  };
  std::vector<Tmp> tmps;

  size_t tmp_top() const { return tmps.empty() ? tmp_base : tmps.back().off + tmps.back().bytes; }
  [[noreturn]] void exhausted(const char* what, size_t need) {
    fail(MM_ENOMEM, std::string("workspace too small for the plan's ") + what + " (" + std::to_string(need) +
                        " bytes past the end of its region; the bound from mm_plan_workspace_size was exceeded)");
  }
  // persistent block (lives as long as the plan)
  template <typename T>
  T* alloc(int64_t count) {
    const size_t b = block_bytes(count, sizeof(T));
    if (pers_top + b > pers_lim) exhausted("persistent data", pers_top + b - pers_lim);
    T* p = reinterpret_cast<T*>(ws + pers_top);
    pers_top += b;
    return p;
  }
  // work vector (from the end of the build on)
  template <typename T>
  T* work(int64_t count) {
    const size_t b = block_bytes(count, sizeof(T));
    if (work_top + b > ws_size) exhausted("work vectors", work_top + b - ws_size);
    T* p = reinterpret_cast<T*>(ws + work_top);
    work_top += b;
    return p;
  }
  // temporary block, released with release(): the stack pops released blocks from its top
  template <typename T>
  T* temp(int64_t count) {
    const size_t b = block_bytes(count, sizeof(T));
    const size_t off = tmp_top();
    if (off + b > ws_size) exhausted("temporaries", off + b - ws_size);
    tmps.push_back(Tmp{off, b, true});
    tmp_peak = std::max(tmp_peak, off + b);
    return reinterpret_cast<T*>(ws + off);
  }
  void release(const void* p) {
    if (!p) return;
    const size_t off = (size_t)((const char*)p - ws);
    for (Tmp& t : tmps)
      if (t.live && t.off == off) t.live = false;
    while (!tmps.empty() && !tmps.back().live) tmps.pop_back();
  }
  // device bytes in use: persistent data, then the larger of the work vectors and the temporaries
  int64_t bytes() const { return (int64_t)(std::max(work_top, tmp_peak)); }

  ~mm_plan_s() {
    for (hipGraphExec_t g : graph)
      if (g) (void)hipGraphExecDestroy(g);   // destructor: statuses are discarded
    // work the caller queued on its own streams may still read the workspace: drain
    // the device before the caller may reuse it
    (void)hipDeviceSynchronize();
    if (ws_owned && ws) (void)hipFree(ws);
    if (st_host) (void)hipHostFree(st_host);
    if (hist_host) (void)hipHostFree(hist_host);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (ev_singular) (void)hipEventDestroy(ev_singular);
    if (ev_ready) (void)hipEventDestroy(ev_ready);
    if (own) stream_put(device, own);
  }

  int64_t nmap() const { return n_obs * ns; }            // map unknowns per RHS
  int64_t vs32() const { return n_obs * ns; }             // row of the float32 copy of p
  // float32 q, z and p in the iteration: mixed precision, no template amplitudes
  bool iter_f32() const { return vp32 != nullptr && !fs_main.fp64 && tmpl.empty(); }
  int64_t nu() const { return n_obs * ns + n_tunk; }     // iteration vector row
  int64_t ng() const { return n_pix * ns + n_tglob; }    // API map-shaped row
  bool main_fp64() const { return precision == MM_FP64; }
};

// preconditioner blocks flagged singular (the count is copied back without a wait
// at plan time and read here when first needed)
int singular_count(mm_plan_s* P) {
  if (P->ev_singular) {
    hipchk(hipEventSynchronize(P->ev_singular), "preconditioner");
    P->n_singular = (int)*P->slot<unsigned long long>(kPinSingular);
    hipchk(hipEventDestroy(P->ev_singular), "event");
    P->ev_singular = nullptr;
  }
  return P->n_singular;
}

namespace {

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// order work on `stream` after the plan's build (the build may have run on another stream)
void wait_ready(mm_plan_s* P, hipStream_t stream) {
  if (P->ev_ready) hipchk(hipStreamWaitEvent(stream, P->ev_ready, 0), "event wait");
}

void build_filter_nf(mm_plan_s* P, FilterSetup& fs, bool fp64, int64_t nf, hipStream_t s, int variant, bool tmp);
void build_symbols(const FilterSetup& fs, const double* lags, int n_filt, int n_c, void* out, char* scr,
                   hipStream_t s);
size_t symbol_scratch_bytes(int logn, bool fp64, int n_filt, int variant = 0);
void apply_ols(mm_plan_s* P, const FilterSetup& fs, bool in_f64, const void* y_in, void* y_out, const void* spec,
               int R, hipStream_t s, const CgState* st = nullptr);

void release_filter(mm_plan_s* P, FilterSetup& fs) {
  P->release(fs.chunks);
  P->release(fs.tw2);
  P->release(fs.ptw);
  P->release(fs.spec);
  P->release(fs.ptw_b);
  P->release(fs.ltab);
  P->release(fs.work);
  fs = FilterSetup();
}

int64_t longest_interval(const std::vector<int64_t>& iv_start) {
  int64_t longest = 1;
  for (size_t b = 0; b + 1 < iv_start.size(); ++b) longest = std::max<int64_t>(longest, iv_start[b + 1] - iv_start[b]);
  return longest;
}

// Transforms of 2^logn complex points: on-chip (one workgroup, workgroup shape v), or
// beyond the on-chip limit the batched four-step transform (one shape, v = 0).
bool transform_long(int logn, bool fp64) { return logn > ols_max_logn(fp64); }
bool transform_exists(int logn, bool fp64, int v) {
  return transform_long(logn, fp64) ? (v == 0 && ols_long_exists(logn)) : ols_variant_exists(logn, fp64, v);
}
constexpr int kMaxLogNLong = 17;   // n_f = 2^18, the paper's length for n_c = 8192

// Lengths the autotuner tries: every power of two above 2 n_c that has a transform (on-chip,
// then the long ones), up to the first whose half already covers twice the longest interval
// (longer ones only add padding).
std::vector<int64_t> autotune_lengths(int n_c, int64_t longest, bool fp64) {
  int64_t nf = 1;
  while (nf <= 2 * (int64_t)n_c) nf <<= 1;
  nf = std::max<int64_t>(nf, int64_t(1) << (kMinLogN + 1));
  std::vector<int64_t> out;
  for (; ilog2(nf) - 1 <= kMaxLogNLong; nf <<= 1) {
    if (transform_exists(ilog2(nf) - 1, fp64, 0)) out.push_back(nf);
    if ((nf >> 1) >= 2 * longest) break;
  }
  if (out.empty()) fail(MM_EUNSUPPORTED, "n_c too large for the transforms");
  return out;
}

// Autotuner: build every admissible on-chip transform (length x workgroup shape) as a
// temporary, time its overlap-save pass over the plan's own intervals, and build the
// fastest one for the plan.
void autotune_filter(mm_plan_s* P, FilterSetup& fs, bool fp64, hipStream_t s) {
  const std::vector<int64_t> lens = autotune_lengths(P->n_c, longest_interval(P->iv_start), fp64);
  hipEvent_t e0, e1;
  hipchk(hipEventCreate(&e0), "event");
  hipchk(hipEventCreate(&e1), "event");
  const int esz = fp64 ? 8 : 4;
  void* ya = P->temp<char>(std::max<int64_t>(P->n_t, 1) * esz);
  void* yb = P->temp<char>(std::max<int64_t>(P->n_t, 1) * esz);
  hipchk(hipMemsetAsync(ya, 0, std::max<int64_t>(P->n_t, 1) * esz, s), "memset");
  float best_ms = 0;
  int64_t best_nf = 0;
  int best_v = 0;
  for (int64_t nf : lens) {
    for (int v = 0; v < kOlsVariants; ++v) {
      if (!transform_exists(ilog2(nf) - 1, fp64, v)) continue;
      FilterSetup cand;
      build_filter_nf(P, cand, fp64, nf, s, v, true);
      apply_ols(P, cand, fp64, ya, yb, cand.spec, 1, s);   // warm-up
      hipchk(hipEventRecord(e0, s), "event");
      for (int rep = 0; rep < 3; ++rep) apply_ols(P, cand, fp64, ya, yb, cand.spec, 1, s);
      hipchk(hipEventRecord(e1, s), "event");
      hipchk(hipEventSynchronize(e1), "autotune");
      float ms = 0;
      hipchk(hipEventElapsedTime(&ms, e0, e1), "event time");
      if (best_nf == 0 || ms < best_ms) {
        best_ms = ms;
        best_nf = nf;
        best_v = v;
      }
      release_filter(P, cand);
    }
  }
  P->release(yb);
  P->release(ya);
  hipchk(hipEventDestroy(e0), "event");
  hipchk(hipEventDestroy(e1), "event");
  build_filter_nf(P, fs, fp64, best_nf, s, best_v, false);
}

// transform shape used when the descriptor leaves it open: the fastest measured
// for each length (2^14 and 2^15 points in float32: the four-step transforms with
// wavefront-private inner stages; 2^14 in float64: 512 threads x 32 points, radix-16
// passes, pairs in registers)
int default_ols_variant(int logn, bool fp64) {
  if (!fp64 && ols_wave_exists(logn, fp64)) return 9;
  return logn == 14 && fp64 ? 2 : 0;
}

int64_t count_chunks(const std::vector<int64_t>& iv_start, int64_t m);

// Compute units of the current device (256 when there is none to ask)
int compute_units() {
  static thread_local int cached_dev = -2, cached_cu = 256;
  int dev = -1, cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  if (dev != cached_dev) {
    cached_dev = dev;
    cached_cu = (dev >= 0 && hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                 cu > 0) ? cu : 256;
  }
  (void)hipGetLastError();
  return cached_cu;
}

// Workgroup time of one 2^15-point wavefront-private transform over one 2^14-point one
// (the float32 filter pass of 2^30 samples x 8 RHS at n_c = 8192: 32.6 ms for 179,088
// jobs at n_f = 2^16 against 42.7 ms for 529,632 at 2^15)
constexpr double kWave15Cost = 2.25;

// n_f of a filter set-up that is not autotuned (secondary: the float64 filter of a
// mixed plan, which takes a forced n_f only when it has a float64 transform).  The
// length rule, capped at 2^14; where that leaves no valid outputs, the smallest power
// of two above 2 n_c, or in float32 with the wavefront-private transforms twice that when
// its chunks (one workgroup each, one workgroup per CU) take less time in full rounds
// over the chip: fewer chunks, no more than 2.25 times the work each.
int64_t choose_nf(int nf_req, int n_c, const std::vector<int64_t>& iv_start, int R, int shape_req, bool fp64,
                  bool secondary) {
  const int maxlog = ols_max_logn(fp64);
  if (nf_req > 0 && !(secondary && ilog2(nf_req) - 1 > maxlog)) return nf_req;
  int64_t nf = fft_length_rule(n_c, longest_interval(iv_start));
  nf = std::min<int64_t>(nf, int64_t(1) << (kPreferredMaxLogN + 1));
  if (nf <= 2 * (int64_t)n_c) {
    nf = 1;
    while (nf <= 2 * (int64_t)n_c) nf <<= 1;
    const bool wave_shape = shape_req == 0 || shape_req == 10;
    if (!fp64 && wave_shape && ilog2(nf) - 1 == 14 && ols_wave_exists(15, false)) {
      const double cu = compute_units();
      auto rounds = [&](int64_t f) {
        return std::ceil((double)count_chunks(iv_start, f - 2 * (int64_t)n_c) * std::max(R, 1) / cu);
      };
      if (kWave15Cost * rounds(2 * nf) < rounds(nf)) nf *= 2;
    }
  }
  return std::max<int64_t>(nf, int64_t(1) << (kMinLogN + 1));
}

int choose_variant(int shape_req, int64_t nf, bool fp64) {
  const int logn = ilog2(nf) - 1;
  const int v = shape_req > 0 ? shape_req - 1 : default_ols_variant(logn, fp64);
  return transform_exists(logn, fp64, v) ? v : 0;
}

void build_filter(mm_plan_s* P, FilterSetup& fs, bool fp64, hipStream_t s, bool secondary = false) {
  if (P->nf_req < 0 && !secondary) {
    autotune_filter(P, fs, fp64, s);
    return;
  }
  const int64_t nf = choose_nf(P->nf_req, P->n_c, P->iv_start, P->R, P->shape_req, fp64, secondary);
  build_filter_nf(P, fs, fp64, nf, s, choose_variant(P->shape_req, nf, fp64), false);
}

int64_t count_chunks(const std::vector<int64_t>& iv_start, int64_t m) {
  int64_t c = 0;
  for (size_t b = 0; b + 1 < iv_start.size(); ++b) c += (iv_start[b + 1] - iv_start[b] + m - 1) / m;
  return c;
}

void check_transform_length(int64_t nf, bool fp64) {
  const int maxlog = ols_max_logn(fp64);
  const int logn = ilog2(nf) - 1;
  if (logn > maxlog && !ols_long_exists(logn))
    fail(MM_EUNSUPPORTED, "no transform of FFT length " + std::to_string(nf) + (fp64 ? " in float64" : " in float32") +
                              " (on-chip up to " + std::to_string(int64_t(1) << (maxlog + 1)) +
                              ", four-step 2^17 and 2^18)");
  if (logn < kMinLogN) fail(MM_EUNSUPPORTED, "FFT length below 128");
}

void build_filter_nf(mm_plan_s* P, FilterSetup& fs, bool fp64, int64_t nf, hipStream_t s, int variant, bool tmp) {
  check_transform_length(nf, fp64);
  const int logn = ilog2(nf) - 1;
  if (!transform_exists(logn, fp64, variant)) variant = 0;
  auto get = [&](int64_t bytes) -> char* { return tmp ? P->temp<char>(bytes) : P->alloc<char>(bytes); };
  fs.fp64 = fp64;
  fs.logn = logn;
  fs.variant = variant;
  fs.N = 1 << logn;
  fs.nf = (int)nf;
  fs.m = fs.nf - 2 * P->n_c;
  if (fs.m <= 0) fail(MM_EINVAL, "n_f must exceed 2 n_c");

  std::vector<OlsChunk>& ch = fs.chunks_host;
  ch.clear();
  for (int b = 0; b < P->n_iv; ++b) {
    const int64_t a = P->iv_start[b], e = P->iv_start[b + 1];
    for (int64_t o = a; o < e; o += fs.m) ch.push_back(OlsChunk{o, a, e, P->iv_filter[b], 0});
  }
  if (ch.size() > (size_t)0x7fffffff) fail(MM_EUNSUPPORTED, "too many overlap-save chunks");
  fs.n_chunks = (int)ch.size();
  fs.chunks = reinterpret_cast<OlsChunk*>(get((int64_t)ch.size() * (int64_t)sizeof(OlsChunk)));
  if (!ch.empty())
    hipchk(hipMemcpyAsync(fs.chunks, ch.data(), ch.size() * sizeof(OlsChunk), hipMemcpyHostToDevice, s),
           "chunk table upload");
  const int esz = fp64 ? 8 : 4;
  fs.tw2 = get((int64_t)fs.N * 2 * esz);
  hipchk(launch_tw2_table(fs.tw2, logn, fp64, s), "twiddle table");
  fs.long_path = transform_long(logn, fp64);
  if (fs.long_path) {   // four-step: twiddles of its 2^8-point columns and 2^(logn - 8)-point rows
    fs.ptw = get((int64_t)std::max(pass_twiddle_count(8, fp64, 0), 1) * 2 * esz);
    hipchk(launch_pass_twiddles(fs.ptw, 8, fp64, s, 0), "pass twiddle tables");
    fs.ptw_b = get((int64_t)std::max(pass_twiddle_count(logn - 8, fp64, 0), 1) * 2 * esz);
    hipchk(launch_pass_twiddles(fs.ptw_b, logn - 8, fp64, s, 0), "pass twiddle tables");
    fs.ltab = get((int64_t)ols_long_table_count(logn) * 2 * esz);
    hipchk(launch_long_tables(logn, fp64, fs.ltab, s), "four-step twiddle tables");
    fs.batch = std::min<int64_t>(ols_long_batch(logn, fp64), std::max<int64_t>((int64_t)fs.n_chunks * P->R, 1));
    fs.work = get(fs.batch * (int64_t)fs.N * 2 * esz);
  } else {
    const int ntw = pass_twiddle_count(logn, fp64, variant);
    if (ntw < 0) fail(MM_EUNSUPPORTED, "no transform for this FFT length");
    fs.ptw = get((int64_t)std::max(ntw, 1) * 2 * esz);
    hipchk(launch_pass_twiddles(fs.ptw, logn, fp64, s, variant), "pass twiddle tables");
  }
  fs.spec = get((int64_t)P->n_filt * (fs.N + 1) * esz);
  char* sscr = P->temp<char>((int64_t)symbol_scratch_bytes(logn, fp64, P->n_filt, fs.variant));
  build_symbols(fs, P->lags, P->n_filt, P->n_c, fs.spec, sscr, s);
  P->release(sscr);   // later work on this stream may reuse it
  fs.ready = true;
}

// Symbol tables F_b / (4N) of n_filt filters from their lags (launch_spectra), in the
// order the transform of fs reads them: natural, or row order for the batched four-step
// transform (launch_long_symbol_rows) and for the wavefront-private one (variant 9,
// launch_wave_symbols); scr: symbol_scratch_bytes
void build_symbols(const FilterSetup& fs, const double* lags, int n_filt, int n_c, void* out, char* scr,
                   hipStream_t s) {
  const bool wave = !fs.long_path && fs.variant == 9;
  if (!fs.long_path && !wave) {
    hipchk(launch_spectra(lags, n_filt, n_c, fs.logn, fs.fp64, out, scr, s), "filter spectra");
    return;
  }
  char* nat = scr + block_bytes((int64_t)spectra_scratch_bytes(fs.logn), 1);
  hipchk(launch_spectra(lags, n_filt, n_c, fs.logn, fs.fp64, nat, scr, s), "filter spectra");
  if (wave)
    hipchk(launch_wave_symbols(fs.logn, nat, out, n_filt, s), "filter spectra in row order");
  else
    hipchk(launch_long_symbol_rows(fs.logn, fs.fp64, nat, out, n_filt, s), "filter spectra in row order");
}

// y_out = N^-1 y_in by the overlap-save transforms of fs with the symbol table spec
// (the plan's filters, or their derivatives); R rows; in_f64 = element type of y_in,
// y_out has the compute type of fs; st (optional): rows of stopped RHS are skipped
void apply_ols(mm_plan_s* P, const FilterSetup& fs, bool in_f64, const void* y_in, void* y_out, const void* spec,
               int R, hipStream_t s, const CgState* st) {
  if (fs.long_path)
    hipchk(launch_ols_long(fs.fp64, in_f64, fs.logn, y_in, y_out, fs.chunks, fs.n_chunks, spec, fs.ptw, fs.ptw_b,
                           fs.tw2, fs.ltab, fs.work, fs.batch, P->n_t, P->n_c, fs.m, R, s, st),
           "overlap-save filter (four-step)");
  else
    hipchk(launch_ols(fs.fp64, in_f64, fs.logn, y_in, y_out, fs.chunks, fs.n_chunks, spec, fs.ptw, fs.tw2, P->n_t,
                      P->n_c, fs.m, R, s, fs.variant, st),
           "overlap-save filter");
}

// y_out = N^-1 y_in with the transforms of fs (or the diagonal f_b(0) when
// n_c = 1); in_f64 = element type of y_in; y_out has the element type of fs
// st (optional): CG states, rows of RHS that stopped iterating are skipped
void weight(mm_plan_s* P, const FilterSetup& fs, const void* y_in, bool in_f64, void* y_out, int R,
            hipStream_t s, const CgState* st = nullptr) {
  if (P->n_c == 1) {
    hipchk(launch_white(fs.fp64, in_f64, P->white_tiles, P->n_white_tiles, P->d_iv_filter, P->lags, P->n_c, y_in,
                        y_out, P->n_t, R, s, st),
           "white-noise weight");
    return;
  }
  apply_ols(P, fs, in_f64, y_in, y_out, fs.spec, R, s, st);
}

// y_r = [P B] x_r: x in iteration layout (rows of stride nu), y a TOD of type y_f64
// x32 (optional): a float32 copy of the map part of x, which the sky gather reads instead
void gather_all(mm_plan_s* P, bool y_f64, const double* x, void* y, int R, hipStream_t s,
                const CgState* st = nullptr, const float* x32 = nullptr) {
  const int64_t vs = P->nu();
  hipchk(launch_gather(y_f64, P->ns, P->px.obs_idx, P->w, x, vs, y, P->n_t, P->n_obs, R, s, st, x32, P->vs32(),
                       P->gather_order),
         "gather");
  for (const Template& T : P->tmpl) {
    const int64_t off = P->nmap() + T.ooff;
    if (T.kind == MM_TMPL_ONEHOT)
      hipchk(launch_onehot_gather(y_f64, T.lay.obs_idx, x, vs, off, y, P->n_t, R, s, st), "template gather");
    else
      hipchk(launch_hwp_gather(y_f64, T.tiles, T.n_tiles, T.d_seg, T.omega, x, vs, off, y, P->n_t, R, s, st),
             "template gather");
  }
}

// refresh the float32 copy of p after p was set outside the iteration kernels
void sync_p32(mm_plan_s* P, hipStream_t s) {
  if (P->vp32) hipchk(launch_rows_to_f32(P->vp, P->nu(), P->vp32, P->vs32(), P->nmap(), P->R, s), "p copy");
}

// q_r = [P B]^T y_r (iteration layout); with p also the p.q partial sums of
// every scatter block in part_pq [R][n_pq]
void scatter_all(mm_plan_s* P, bool y_f64, const void* y, double* q, int R, hipStream_t s,
                 const double* p = nullptr, const CgState* st = nullptr) {
  const int64_t vs = P->nu();
  hipchk(launch_scatter(y_f64, P->ns, P->px.sell, y, q, vs, P->n_obs, P->n_t, R, s, p, P->part_pq, P->n_pq, 0, st),
         "scatter");
  for (const Template& T : P->tmpl) {
    const int64_t off = P->nmap() + T.ooff;
    if (T.kind == MM_TMPL_ONEHOT) {
      if (T.lay.n_obs == 0) continue;
      hipchk(launch_scatter(y_f64, 1, T.lay.sell, y, q + off, vs, T.lay.n_obs, P->n_t, R, s, p ? p + off : nullptr,
                            P->part_pq, P->n_pq, T.pq_slot, st),
             "template scatter");
    } else {
      hipchk(launch_hwp_scatter(y_f64, T.tiles, T.n_tiles, T.d_seg_tile, T.n_seg, T.d_seg, T.omega, y, P->n_t, R,
                                T.partial, q, vs, off, p, P->part_pq, P->n_pq, T.pq_slot, s, st),
             "template scatter");
    }
  }
}

// API map-shaped rows (stride ng, global ids) <-> iteration rows (stride nu, observed ids)
void to_obs(mm_plan_s* P, const double* glob, double* obs, int R, hipStream_t s) {
  hipchk(launch_to_observed(glob, P->ng(), obs, P->nu(), P->px.obs2glob, P->n_obs, P->n_pix, P->ns, R, s), "layout");
  for (const Template& T : P->tmpl) {
    const double* g = glob + P->n_pix * P->ns + T.goff;
    double* o = obs + P->nmap() + T.ooff;
    if (T.kind == MM_TMPL_ONEHOT)
      hipchk(launch_to_observed(g, P->ng(), o, P->nu(), T.lay.obs2glob, T.lay.n_obs, T.n_glob, 1, R, s), "layout");
    else
      hipchk(launch_copy_rows(g, P->ng(), o, P->nu(), T.n_unk, R, s), "layout");
  }
}

void to_glob(mm_plan_s* P, const double* obs, double* glob, int R, hipStream_t s) {
  hipchk(launch_to_global(obs, P->nu(), glob, P->ng(), P->px.obs2glob, P->n_obs, P->n_pix, P->ns, R, s), "layout");
  for (const Template& T : P->tmpl) {
    double* g = glob + P->n_pix * P->ns + T.goff;
    const double* o = obs + P->nmap() + T.ooff;
    if (T.kind == MM_TMPL_ONEHOT)
      hipchk(launch_to_global(o, P->nu(), g, P->ng(), T.lay.obs2glob, T.lay.n_obs, T.n_glob, 1, R, s), "layout");
    else
      hipchk(launch_copy_rows(o, P->nu(), g, P->ng(), T.n_unk, R, s), "layout");
  }
}

// out = [P B]^T N^-1 [P B] in (iteration layout), R right-hand sides, precision of fs
void apply_H_obs(mm_plan_s* P, const FilterSetup& fs, const double* in, double* out, void* ya, void* yb,
                 int R, hipStream_t s) {
  gather_all(P, fs.fp64, in, ya, R, s);
  weight(P, fs, ya, fs.fp64, yb, R, s);
  scatter_all(P, fs.fp64, yb, out, R, s);
}

void rhs_obs(mm_plan_s* P, const FilterSetup& fs, const void* tod, bool tod_f64, double* out, void* yb,
             int R, hipStream_t s) {
  weight(P, fs, tod, tod_f64, yb, R, s);
  scatter_all(P, fs.fp64, yb, out, R, s);
}


void check_tod_dtype(int32_t dt) {
  if (dt != MM_F32 && dt != MM_F64) fail(MM_EINVAL, "tod_dtype must be MM_F32 or MM_F64");
}

// Largest TOD one scatter pass reads (rows of up to 4 RHS) for which the pixel-major
// scatter is used.  A TOD cache line holds hits of several neighbouring pixels,
// which that scatter reads from different wavefronts (the sliced one from one):
// measured faster while those re-reads mostly stay in the 256 MiB last-level
// cache (64 MiB of float32 TOD: 7 % less time per iteration; 128 MiB of float64
// TOD: 4 % less; 4 RHS x 64 MiB: 6 % less) and slower beyond it (512 MiB: 6 %
// more; 1 GiB: 5 % more).
constexpr int64_t kSegTodBytes = int64_t(256) << 20;

// Wavefronts per slice of the scatter over a layout (0 = no slices: the scatter reads
// the pixel-major arrays as they are)
int layout_waves(int64_t n_t, bool fp64, int R, int64_t n_obs, int64_t n_valid) {
  int wps = scatter_waves_per_slice(n_obs > 0 ? (double)n_valid / (double)n_obs : 1.0);
  const int64_t pass_bytes = n_t * (fp64 ? 8 : 4) * std::min(R, 4);
  if (wps == 0 && pass_bytes > kSegTodBytes) wps = 8;
  return wps;
}

// Entries the sliced copy of a layout with n_valid samples may take (padding to the
// widest pixel of each slice included); a layout whose slices need more keeps the
// pixel-major arrays for the scatter.  Bounds the workspace from the descriptor alone.
int64_t sliced_allowance(int64_t n_valid) { return (2 * n_valid / 64 + 1) * 64; }

// Pixel-major layout of a pointing with one non-zero per row: range check,
// stable sort of the samples by key, observed compaction (Implementation
// section, observed index scheme).  Keys lie in [-1, n_keys); -1 = no column.
// The pixel-major sample ids and weights are temporaries when the scatter will
// read a sliced copy of them (build_sell), else they are kept.
void build_layout(mm_plan_s* P, const int32_t* d_key, int64_t n_keys, int ns, const float* d_w, Layout& L,
                  hipStream_t s, const char* range_msg) {
  const int64_t n = P->n_t;
  // The range check is read at the first synchronisation below: the sort and the
  // layout kernels stay in bounds whatever the indices (an index outside the range
  // only misplaces its sample, and the plan fails before anything uses the result).
  int32_t* flag = P->temp<int32_t>(1);
  hipchk(launch_fill_i32(flag, 0, 1, s), "fill");
  hipchk(launch_check_pix(d_key, n, n_keys, flag, s), "index check");
  L.obs_idx = P->alloc<int32_t>(n);
  L.wps = 0;
  if (n == 0) {
    hipchk(hipMemcpyAsync(P->slot<int32_t>(kPinFlag), flag, 4, hipMemcpyDeviceToHost, s), "index check copy");
    hipchk(hipStreamSynchronize(s), "index check");
    if (*P->slot<int32_t>(kPinFlag)) fail(MM_EINVAL, range_msg);
  }
  if (n > 0) {
    char* scratch = P->temp<char>((int64_t)sort_scratch_bytes(n));
    uint32_t* keys = P->temp<uint32_t>(n);
    int32_t* vals = P->temp<int32_t>(n);
    hipchk(launch_sort_by_pixel(d_key, n, n_keys, keys, vals, scratch, s), "sort by pixel");
    P->release(scratch);
    uint32_t* seg = P->temp<uint32_t>(n);
    char* sscr = P->temp<char>((int64_t)scan_scratch_bytes(n));
    int64_t* nvalid_d = P->temp<int64_t>(1);
    hipchk(hipMemsetAsync(nvalid_d, 0, sizeof(int64_t), s), "memset");
    hipchk(launch_segment_scan(keys, n, (uint32_t)n_keys, seg, nvalid_d, sscr, s), "observed ids");
    hipchk(hipMemcpyAsync(P->slot<int32_t>(kPinFlag), flag, 4, hipMemcpyDeviceToHost, s), "index check copy");
    hipchk(hipMemcpyAsync(P->slot<uint32_t>(kPinObs), seg + (n - 1), 4, hipMemcpyDeviceToHost, s), "copy");
    hipchk(hipMemcpyAsync(P->slot<int64_t>(kPinValid), nvalid_d, 8, hipMemcpyDeviceToHost, s), "copy");
    hipchk(hipStreamSynchronize(s), "observed count");
    if (*P->slot<int32_t>(kPinFlag)) fail(MM_EINVAL, range_msg);
    L.n_obs = *P->slot<uint32_t>(kPinObs);
    L.n_valid = *P->slot<int64_t>(kPinValid);
    L.wps = layout_waves(n, P->main_fp64(), P->R, L.n_obs, L.n_valid);
    L.ptr = P->alloc<int64_t>(L.n_obs + 1);
    L.obs2glob = P->alloc<int32_t>(L.n_obs);
    if (L.wps > 0) {
      L.perm = P->temp<int32_t>(L.n_valid);
      if (ns == 3) L.w_pm = P->temp<float>(2 * L.n_valid);
    } else {
      L.perm = P->alloc<int32_t>(L.n_valid);
      if (ns == 3) L.w_pm = P->alloc<float>(2 * L.n_valid);
    }
    hipchk(launch_build_layout(keys, vals, seg, n, (uint32_t)n_keys, d_w, ns, L.ptr, L.obs2glob, L.w_pm, L.perm, s),
           "pointing layout");
    int32_t* glob2obs = P->temp<int32_t>(n_keys);
    hipchk(launch_obs_index(d_key, n, L.obs2glob, L.n_obs, glob2obs, n_keys, L.obs_idx, s), "observed index");
    P->release(glob2obs);
    hipchk(hipMemcpyAsync(L.ptr + L.n_obs, &L.n_valid, 8, hipMemcpyHostToDevice, s), "copy");
    // released blocks are only reused by later work on this stream: no wait needed
    P->release(keys);
    P->release(vals);
    P->release(seg);
    P->release(sscr);
    P->release(nvalid_d);
  } else {
    L.ptr = P->alloc<int64_t>(1);
    hipchk(hipMemsetAsync(L.ptr, 0, 8, s), "memset");
    L.obs2glob = P->alloc<int32_t>(1);
    L.perm = P->alloc<int32_t>(1);
  }
  P->release(flag);
  const double avg = L.n_obs > 0 ? (double)L.n_valid / (double)L.n_obs : 1.0;
  int g = 4;
  while (g < 64 && g * 4 < avg) g *= 2;
  L.group = g;
}

// Map bytes one gather pass looks up (all RHS) above which the gather visits its tiles
// sorted by pixel rather than in time order: beyond one XCD's 4 MiB L2, the pixels a
// scan revisits (other detectors, later passes) are gone from the caches by then in
// time order, while sorted tiles that see the same pixels run together on one XCD.
constexpr int64_t kGatherOrderMapBytes = int64_t(4) << 20;

// Gather order: the gather tiles sorted (stably) by the smallest observed id each sees.
void build_gather_order(mm_plan_s* P, hipStream_t s) {
  const int64_t map_bytes = P->n_obs * P->ns * (P->main_fp64() ? 8 : 4) * (int64_t)P->R;
  if (P->n_obs == 0 || map_bytes <= kGatherOrderMapBytes) return;
  const int64_t n_tiles = gather_tiles(P->n_t);
  int32_t* key = P->temp<int32_t>(n_tiles);
  hipchk(launch_tile_keys(P->px.obs_idx, P->n_t, key, s), "gather tile keys");
  uint32_t* sorted = P->temp<uint32_t>(n_tiles);
  char* scr = P->temp<char>((int64_t)sort_scratch_bytes(n_tiles));
  P->gather_order = P->alloc<int32_t>(n_tiles);
  hipchk(launch_sort_by_pixel(key, n_tiles, P->n_obs, sorted, P->gather_order, scr, s), "gather order");
  P->release(scr);
  P->release(sorted);
  P->release(key);
}

// The scatter's view of a layout: the pixel-major arrays as they are (L.wps = 0), or
// a sliced copy that replaces them.  A copy that would exceed sliced_allowance
// entries is not made: the pixel-major arrays are kept instead.
void build_sell(mm_plan_s* P, Layout& L, int ns, hipStream_t s) {
  auto keep_pixel_major = [&]() {
    L.sell_entries = L.n_valid;
    L.sell.wps = 0;
    L.sell.ptr = L.ptr;
    L.sell.perm = L.perm;
    L.sell.w_pm = L.w_pm;
  };
  if (L.wps == 0) {   // pixels with many hits: the scatter reads the pixel-major arrays as they are
    keep_pixel_major();
    return;
  }
  const int64_t n_sl = (L.n_obs + 63) / 64;
  uint32_t* len = P->alloc<uint32_t>(n_sl);
  uint32_t* end = P->alloc<uint32_t>(n_sl);
  char* sscr = P->temp<char>((int64_t)scan_scratch_bytes(std::max<int64_t>(n_sl, 1)));
  uint32_t total = 0;
  bool fits = true;
  if (n_sl > 0) {
    hipchk(launch_sell_widths(L.ptr, L.n_obs, len, s), "slice widths");
    hipchk(launch_scan_inclusive(len, end, n_sl, sscr, s), "slice offsets");
    hipchk(hipMemcpyAsync(P->slot<uint32_t>(kPinTotal), end + (n_sl - 1), 4, hipMemcpyDeviceToHost, s), "copy");
    hipchk(hipStreamSynchronize(s), "slices");
    total = *P->slot<uint32_t>(kPinTotal);
    // the 32-bit slice sizes and their prefix sum are exact while the padded total
    // stays below 2^32 - 1 (a saturated size also trips this test).  A slice holds at
    // most 64 x its pixels' hits, so the total is at most 64 n_valid: only larger
    // layouts need the sizes summed exactly.
    if (64.0 * (double)L.n_valid >= 4294967295.0) {
      double check = 0;
      std::vector<uint32_t> hl(n_sl);
      hipchk(hipMemcpy(hl.data(), len, 4 * n_sl, hipMemcpyDeviceToHost), "copy");
      for (uint32_t v : hl) check += v;
      if (check >= 4294967295.0) fits = false;
    }
    if ((int64_t)total > sliced_allowance(L.n_valid)) fits = false;
  }
  P->release(sscr);
  if (!fits) {
    // move the pixel-major arrays out of the temporaries and scatter over them
    int32_t* perm = P->alloc<int32_t>(L.n_valid);
    hipchk(hipMemcpyAsync(perm, L.perm, 4 * L.n_valid, hipMemcpyDeviceToDevice, s), "copy");
    P->release(L.perm);
    L.perm = perm;
    if (ns == 3) {
      float* w = P->alloc<float>(2 * L.n_valid);
      hipchk(hipMemcpyAsync(w, L.w_pm, 8 * L.n_valid, hipMemcpyDeviceToDevice, s), "copy");
      P->release(L.w_pm);
      L.w_pm = w;
    }
    L.wps = 0;
    keep_pixel_major();
    return;
  }
  L.sell_entries = total;
  int32_t* st = P->alloc<int32_t>(std::max<int64_t>(total, 1));
  float* sw = ns == 3 ? P->alloc<float>(2 * std::max<int64_t>(total, 1)) : nullptr;
  hipchk(launch_sell_fill(L.ptr, L.perm, L.w_pm, L.n_obs, end, len, st, sw, ns, s), "slice fill");
  L.sell.end = end;
  L.sell.len = len;
  L.sell.t = st;
  L.sell.w = sw;
  L.sell.wps = L.wps;
  P->release(L.w_pm);
  L.w_pm = nullptr;
  P->release(L.perm);
  L.perm = nullptr;
}

// Validate the descriptor's templates and build their layouts ("Using MADmap" section).
// host-side checks of the template descriptors (before any device work)
void validate_templates(const mm_desc_t* d) {
  if (d->n_templates < 0 || d->n_templates > 16) fail(MM_EINVAL, "n_templates must be in [0, 16]");
  if (d->n_templates > 0 && !d->templates) fail(MM_EINVAL, "templates is NULL");
  for (int k = 0; k < d->n_templates; ++k) {
    const mm_template_t& D = d->templates[k];
    if (D.kind == MM_TMPL_ONEHOT) {
      if (D.n_amp < 1 || D.n_amp >= (int64_t(1) << 31) - 1) fail(MM_EINVAL, "template n_amp must be in [1, 2^31 - 1)");
      if (d->n_samples > 0 && !D.d_idx) fail(MM_EINVAL, "template d_idx is NULL");
    } else if (D.kind == MM_TMPL_HWP) {
      if (D.n_seg < 1 || !D.seg_start) fail(MM_EINVAL, "HWP template needs n_seg >= 1 and seg_start");
      if (d->n_samples > 0 && !D.d_omega) fail(MM_EINVAL, "template d_omega is NULL");
      if (D.seg_start[0] != 0 || D.seg_start[D.n_seg] != d->n_samples)
        fail(MM_EINVAL, "HWP segments must start at 0 and end at n_samples");
      for (int g = 0; g < D.n_seg; ++g)
        if (D.seg_start[g + 1] < D.seg_start[g]) fail(MM_EINVAL, "seg_start must be non-decreasing");
    } else {
      fail(MM_EINVAL, "unknown template kind");
    }
  }
}

void setup_templates(mm_plan_s* P, const mm_desc_t* d, hipStream_t s) {
  P->tmpl.resize(d->n_templates);
  int64_t goff = 0, ooff = 0;
  for (int k = 0; k < d->n_templates; ++k) {
    const mm_template_t& D = d->templates[k];
    Template& T = P->tmpl[k];
    T.kind = D.kind;
    if (D.kind == MM_TMPL_ONEHOT) {
      build_layout(P, D.d_idx, D.n_amp, 1, nullptr, T.lay, s, "template index outside [-1, n_amp)");
      T.n_glob = D.n_amp;
      T.n_unk = T.lay.n_obs;
    } else {
      T.omega = D.d_omega;
      T.n_seg = D.n_seg;
      T.seg_host.assign(D.seg_start, D.seg_start + D.n_seg + 1);
      std::vector<SampleTile> tiles;
      std::vector<int32_t> first(D.n_seg + 1);
      for (int g = 0; g < D.n_seg; ++g) {
        first[g] = (int32_t)std::min<size_t>(tiles.size(), 0x7fffffff);
        for (int64_t t0 = T.seg_host[g]; t0 < T.seg_host[g + 1]; t0 += kTileSamples)
          tiles.push_back(SampleTile{t0, std::min<int64_t>(t0 + kTileSamples, T.seg_host[g + 1]), g, 0});
      }
      if (tiles.size() > (size_t)0x7fffffff) fail(MM_EUNSUPPORTED, "too many template tiles");
      first[D.n_seg] = (int32_t)tiles.size();
      T.n_tiles = (int)tiles.size();
      T.tiles = P->alloc<SampleTile>(std::max<int64_t>(T.n_tiles, 1));
      T.d_seg = P->alloc<int64_t>(D.n_seg + 1);
      T.d_seg_tile = P->alloc<int32_t>(D.n_seg + 1);
      T.partial = P->alloc<double>((int64_t)std::max(T.n_tiles, 1) * P->R * kHwpColumns);
      if (T.n_tiles > 0)
        hipchk(hipMemcpyAsync(T.tiles, tiles.data(), tiles.size() * sizeof(SampleTile), hipMemcpyHostToDevice, s),
               "tile upload");
      hipchk(hipMemcpyAsync(T.d_seg, T.seg_host.data(), 8 * (D.n_seg + 1), hipMemcpyHostToDevice, s), "copy");
      hipchk(hipMemcpyAsync(T.d_seg_tile, first.data(), 4 * (D.n_seg + 1), hipMemcpyHostToDevice, s), "copy");
      hipchk(hipStreamSynchronize(s), "template tiles");
      T.n_glob = T.n_unk = (int64_t)kHwpColumns * D.n_seg;
    }
    T.goff = goff;
    T.ooff = ooff;
    goff += T.n_glob;
    ooff += T.n_unk;
  }
  P->n_tglob = goff;
  P->n_tunk = ooff;
}

// Coarse index of the interval table for sample -> interval lookups on the device:
// hint[c] = the last interval starting at or before sample c << shift.  Buckets are
// no longer than the shortest non-empty interval (while the table stays within 2^20
// entries), so a sample lies at most a few interval starts past its bucket's hint.
int interval_hint_shift(const std::vector<int64_t>& iv_start, int64_t n_t) {
  int64_t lmin = std::max<int64_t>(n_t, 1);
  for (size_t b = 0; b + 1 < iv_start.size(); ++b) {
    const int64_t len = iv_start[b + 1] - iv_start[b];
    if (len > 0) lmin = std::min(lmin, len);
  }
  int sh = 0;
  while ((int64_t(2) << sh) <= lmin) ++sh;
  while ((n_t >> sh) + 1 > (int64_t(1) << 20)) ++sh;
  return sh;
}

void build_interval_hint(mm_plan_s* P, hipStream_t s) {
  const int sh = interval_hint_shift(P->iv_start, P->n_t);
  const int64_t nb = (P->n_t >> sh) + 1;
  std::vector<int32_t>& hint = P->iv_hint;
  hint.assign((size_t)nb, 0);
  int b = 0;
  for (int64_t c = 0; c < nb; ++c) {
    const int64_t t0 = c << sh;
    while (b + 1 < P->n_iv && P->iv_start[b + 1] <= t0) ++b;
    hint[(size_t)c] = b;
  }
  P->iv_hint_shift = sh;
  P->d_iv_hint = P->alloc<int32_t>(nb);
  hipchk(hipMemcpyAsync(P->d_iv_hint, hint.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, s), "copy");
}

// Diagonal preconditioner of the template amplitudes: diag(B^T W^-1 B)^-1
// (block), diag(B^T B)^-1 (Jacobi) or 1; 0 for an all-zero column.
void build_template_precond(mm_plan_s* P, hipStream_t s) {
  P->minv_t = P->alloc<double>(std::max<int64_t>(P->n_tunk, 1));
  for (Template& T : P->tmpl) {
    double* dst = P->minv_t + T.ooff;
    if (T.kind == MM_TMPL_ONEHOT) {
      if (T.lay.n_obs == 0) continue;
      int32_t* sing = P->temp<int32_t>(T.lay.n_obs);
      hipchk(launch_precond_build(1, P->precond, T.lay.group, T.lay.ptr, T.lay.perm, nullptr, P->d_iv_start,
                                  P->n_iv, P->d_iv_hint, P->iv_hint_shift, P->d_iv_filter, P->lags, P->n_c,
                                  T.lay.n_obs, dst, sing, s),
             "template preconditioner");
      hipchk(hipStreamSynchronize(s), "template preconditioner");
      P->release(sing);
    } else if (P->precond == MM_PRECOND_NONE) {
      hipchk(launch_fill_f64(dst, 1.0, T.n_unk, s), "fill");
    } else {
      double* diag = P->temp<double>(T.n_unk);
      hipchk(launch_hwp_diag(P->precond == MM_PRECOND_BLOCK ? 0 : 1, T.tiles, T.n_tiles, T.d_seg_tile, T.n_seg,
                             T.d_seg, T.omega, P->d_iv_start, P->n_iv, P->d_iv_filter, P->lags, P->n_c, T.partial,
                             diag, s),
             "template preconditioner");
      hipchk(launch_invert_diag(diag, dst, T.n_unk, s), "template preconditioner");
      hipchk(hipStreamSynchronize(s), "template preconditioner");
      P->release(diag);
    }
  }
}

// Host-side checks of a descriptor (before any device work); the interval table
// and filter parameters are checked as well.
void validate_desc(const mm_desc_t* d) {
  if (!d) fail(MM_EINVAL, "descriptor is NULL");
  if (d->n_stokes != 1 && d->n_stokes != 3) fail(MM_EINVAL, "n_stokes must be 1 or 3");
  if (d->n_pix < 1 || d->n_pix >= (int64_t(1) << 31) - 1) fail(MM_EINVAL, "n_pix must be in [1, 2^31 - 1)");
  if (d->n_samples < 0 || d->n_samples > (int64_t(1) << 31) - 1)
    fail(MM_EINVAL, "n_samples must be in [0, 2^31 - 1]");
  if (d->n_intervals < 1 || !d->iv_start || !d->iv_filter) fail(MM_EINVAL, "interval table missing");
  if (d->n_filters < 1) fail(MM_EINVAL, "n_filters must be >= 1");
  if (d->n_c < 1) fail(MM_EINVAL, "n_c must be >= 1");
  if (!d->filter_params && !d->filter_lags) fail(MM_EINVAL, "give filter_params or filter_lags");
  if (d->precision != MM_FP64 && d->precision != MM_MIXED) fail(MM_EINVAL, "precision must be MM_FP64 or MM_MIXED");
  if (d->precond < MM_PRECOND_BLOCK || d->precond > MM_PRECOND_NONE) fail(MM_EINVAL, "unknown preconditioner");
  if (d->n_rhs < 1 || d->n_rhs > 64) fail(MM_EINVAL, "n_rhs must be in [1, 64]");
  if (d->n_f != 0 && d->n_f != -1 && (!is_pow2(d->n_f) || d->n_f <= 2 * d->n_c))
    fail(MM_EINVAL, "n_f must be 0, -1 or a power of two above 2 n_c");
  if (d->fft_shape < 0 || d->fft_shape > kOlsVariants) fail(MM_EINVAL, "fft_shape must be in [0, 10]");
  validate_templates(d);
  if (d->iv_start[0] != 0 || d->iv_start[d->n_intervals] != d->n_samples)
    fail(MM_EINVAL, "intervals must start at 0 and end at n_samples");
  for (int b = 0; b < d->n_intervals; ++b) {
    if (d->iv_start[b + 1] < d->iv_start[b]) fail(MM_EINVAL, "iv_start must be non-decreasing");
    if (d->iv_filter[b] < 0 || d->iv_filter[b] >= d->n_filters) fail(MM_EINVAL, "iv_filter out of range");
  }
  const int ncp = 1 << std::max(kMinLogN, ilog2(d->n_c));
  const int64_t lag_len = d->lag_dft_len ? d->lag_dft_len : (1 << 20);
  if (d->filter_params) {
    if (!(d->f_samp > 0)) fail(MM_EINVAL, "f_samp must be positive");
    if (!is_pow2(lag_len) || lag_len < 4 * (int64_t)ncp) fail(MM_EINVAL, "lag_dft_len must be a power of two >= 4 n_c");
    if (ncp > (1 << ols_max_logn(true))) fail(MM_EUNSUPPORTED, "n_c too large for the lag construction");
    for (int f = 0; f < d->n_filters; ++f) {
      const double sg = d->filter_params[3 * f], fk = d->filter_params[3 * f + 1], al = d->filter_params[3 * f + 2];
      if (!(sg > 0) || !(fk >= 0) || !(al > 0) || !std::isfinite(sg) || !std::isfinite(fk) || !std::isfinite(al))
        fail(MM_EINVAL, "filter parameters need sigma > 0, f_knee >= 0, alpha > 0");
    }
  }
}

int64_t y_bytes(bool fp64, int R, int64_t n) { return fp64 ? (int64_t)R * n * 8 : std::max<int64_t>((int64_t)R * 4, 8) * n; }

// Scratch of build_symbols: the spectra's own, then (four-step transform) the tables in
// natural order before they are put in row order
size_t symbol_scratch_bytes(int logn, bool fp64, int n_filt, int variant) {
  const size_t b = spectra_scratch_bytes(logn);
  if (!transform_long(logn, fp64) && !(variant == 9 && ols_wave_exists(logn, fp64))) return b;
  return block_bytes((int64_t)b, 1) + (size_t)n_filt * ((size_t(1) << logn) + 1) * (fp64 ? 8 : 4);
}

// Device bytes of a filter set-up (chunk table, twiddles, spectra) and of the
// spectra build's scratch
size_t filter_bytes(const std::vector<int64_t>& iv_start, int n_filt, int n_c, int64_t nf, int variant, bool fp64,
                    int R) {
  const int logn = ilog2(nf) - 1;
  const int64_t N = int64_t(1) << logn;
  const int esz = fp64 ? 8 : 4;
  const int64_t n_chunks = count_chunks(iv_start, nf - 2 * n_c);
  size_t tw;
  if (transform_long(logn, fp64)) {   // column and row twiddles, intermediates of a batch
    const int64_t batch = std::min<int64_t>(ols_long_batch(logn, fp64), std::max<int64_t>(n_chunks * R, 1));
    tw = block_bytes((int64_t)std::max(pass_twiddle_count(8, fp64, 0), 1) * 2 * esz, 1) +
         block_bytes((int64_t)std::max(pass_twiddle_count(logn - 8, fp64, 0), 1) * 2 * esz, 1) +
         block_bytes((int64_t)ols_long_table_count(logn) * 2 * esz, 1) + block_bytes(batch * N * 2 * esz, 1);
  } else {
    tw = block_bytes((int64_t)std::max(pass_twiddle_count(logn, fp64, variant), 1) * 2 * esz, 1);
  }
  return block_bytes(n_chunks * (int64_t)sizeof(OlsChunk), 1) + block_bytes(N * 2 * esz, 1) + tw +
         block_bytes((int64_t)n_filt * (N + 1) * esz, 1);
}

// Upper bounds of a plan's device memory from its descriptor alone: persistent data,
// work vectors, the build's temporaries (stacked over the work region) and the
// temporaries of later calls (stacked above the TOD work buffers).  Every count the
// data decide is bounded: observed pixels by min(n_pix, n_samples) (one-hot
// amplitudes by min(n_amp, n_samples)), pointed samples by n_samples, a sliced
// scatter layout by sliced_allowance, the p.q partial sums by kScatterBlocks per
// scatter.
struct PlanBounds {
  size_t pers = 0, work = 0, temps = 0, call_temps = 0;
  size_t total() const { return pers + std::max(work + call_temps, temps) + kAlign; }
};

PlanBounds plan_bounds(const mm_desc_t* d) {
  validate_desc(d);
  PlanBounds B;
  const int64_t n = d->n_samples;
  const int ns = d->n_stokes, R = d->n_rhs, nf_filt = d->n_filters, n_c = d->n_c;
  const bool fp64 = d->precision == MM_FP64;
  const std::vector<int64_t> iv(d->iv_start, d->iv_start + d->n_intervals + 1);
  const int64_t longest = longest_interval(iv);
  // pixel-major layout of a pointing with one non-zero per row (build_layout, build_sell)
  auto layout = [&](int64_t n_keys, int lns, int64_t* n_obs_out) {
    const int64_t n_obs = std::min<int64_t>(n_keys, n);
    *n_obs_out = n_obs;
    B.pers += block_bytes(n, 4);
    B.temps += block_bytes(1, 4);
    if (n == 0) {
      B.pers += block_bytes(1, 8) + 2 * block_bytes(1, 4);
      return;
    }
    const int64_t n_sl = (n_obs + 63) / 64;
    const int64_t allow = sliced_allowance(n);
    const size_t csr = block_bytes(n, 4) + (lns == 3 ? block_bytes(2 * n, 4) : 0);
    const size_t sliced = block_bytes(allow, 4) + (lns == 3 ? block_bytes(2 * allow, 4) : 0);
    B.pers += block_bytes(n_obs + 1, 8) + block_bytes(n_obs, 4) + 2 * block_bytes(n_sl, 4) + std::max(csr, sliced);
    B.temps += block_bytes((int64_t)sort_scratch_bytes(n), 1) + 3 * block_bytes(n, 4) +
               block_bytes((int64_t)scan_scratch_bytes(n), 1) + block_bytes(1, 8) + csr + block_bytes(n_keys, 4) +
               block_bytes((int64_t)scan_scratch_bytes(std::max<int64_t>(n_sl, 1)), 1);
  };
  int64_t n_obs = 0;
  layout(d->n_pix, ns, &n_obs);
  {   // gather order (build_gather_order)
    const int64_t n_tiles = gather_tiles(n);
    B.pers += block_bytes(n_tiles, 4);
    B.temps += 2 * block_bytes(n_tiles, 4) + block_bytes((int64_t)sort_scratch_bytes(n_tiles), 1);
  }
  int64_t n_tunk = 0, n_pq = n_obs > 0 ? kScatterBlocks : 0;
  for (int k = 0; k < d->n_templates; ++k) {
    const mm_template_t& D = d->templates[k];
    if (D.kind == MM_TMPL_ONEHOT) {
      int64_t n_amp_obs = 0;
      layout(D.n_amp, 1, &n_amp_obs);
      n_tunk += n_amp_obs;
      n_pq += kScatterBlocks;
      B.temps += block_bytes(n_amp_obs, 4);                       // preconditioner flags
    } else {
      int64_t n_tiles = 0;
      for (int g = 0; g < D.n_seg; ++g) n_tiles += (D.seg_start[g + 1] - D.seg_start[g] + kTileSamples - 1) / kTileSamples;
      B.pers += block_bytes(n_tiles, sizeof(SampleTile)) + block_bytes(D.n_seg + 1, 8) + block_bytes(D.n_seg + 1, 4) +
                block_bytes(std::max<int64_t>(n_tiles, 1) * R * kHwpColumns, 8);
      n_tunk += (int64_t)kHwpColumns * D.n_seg;
      n_pq += 1;
      B.temps += block_bytes((int64_t)kHwpColumns * D.n_seg, 8);  // preconditioner diagonal
    }
  }
  // noise filters
  const int64_t lag_len = d->lag_dft_len ? d->lag_dft_len : (1 << 20);
  const int batch = std::max(1, std::min(nf_filt, 16));
  B.pers += block_bytes((int64_t)nf_filt * n_c, 8);
  if (d->filter_params) {
    B.pers += block_bytes(3 * (int64_t)nf_filt, 8);
    B.temps += block_bytes((int64_t)lags_scratch_bytes(n_c, lag_len, batch), 1);
  }
  int logn64 = 0;   // transform of the float64 filter (noise gradient)
  if (d->n_f < 0) {
    size_t most = 0, most_tmp = 0;
    for (int64_t nf : autotune_lengths(n_c, longest, fp64))
      for (int v = 0; v < kOlsVariants; ++v) {
        if (!transform_exists(ilog2(nf) - 1, fp64, v)) continue;
        const size_t fb = filter_bytes(iv, nf_filt, n_c, nf, v, fp64, R);
        most = std::max(most, fb);
        most_tmp =
            std::max(most_tmp, fb + block_bytes((int64_t)symbol_scratch_bytes(ilog2(nf) - 1, fp64, nf_filt, v), 1));
        if (fp64) logn64 = std::max(logn64, ilog2(nf) - 1);
      }
    B.pers += most;
    B.temps += 2 * block_bytes(std::max<int64_t>(n, 1) * (fp64 ? 8 : 4), 1) + most_tmp + most;
  } else {
    const int64_t nf = choose_nf(d->n_f, n_c, iv, R, d->fft_shape, fp64, false);
    const int logn = ilog2(nf) - 1;
    check_transform_length(nf, fp64);
    const int v = choose_variant(d->fft_shape, nf, fp64);
    B.pers += filter_bytes(iv, nf_filt, n_c, nf, v, fp64, R);
    B.temps += block_bytes((int64_t)symbol_scratch_bytes(logn, fp64, nf_filt, v), 1);
    if (fp64) logn64 = logn;
  }
  if (!fp64) {
    const int64_t nf = choose_nf(d->n_f, n_c, iv, R, d->fft_shape, true, true);
    logn64 = ilog2(nf) - 1;
    check_transform_length(nf, true);
    B.pers += filter_bytes(iv, nf_filt, n_c, nf, choose_variant(d->fft_shape, nf, true), true, R);
    B.temps += block_bytes((int64_t)symbol_scratch_bytes(logn64, true, nf_filt), 1);
  }
  // interval tables and their coarse index
  const int sh = interval_hint_shift(iv, n);
  B.pers += block_bytes(d->n_intervals + 1, 8) + block_bytes(d->n_intervals, 4) + block_bytes((n >> sh) + 1, 4);
  // preconditioner
  B.pers += block_bytes(n_obs * (ns == 1 ? 1 : 6), 8) + block_bytes(std::max<int64_t>(n_tunk, 1), 8);
  B.temps += block_bytes(n_obs, 4) + block_bytes(1, 8);
  if (n_c == 1) {
    int64_t n_wt = 0;
    for (int b = 0; b < d->n_intervals; ++b) n_wt += (iv[b + 1] - iv[b] + kTileSamples - 1) / kTileSamples;
    B.pers += block_bytes(n_wt, sizeof(SampleTile));
  }
  // scalars, partial sums, residual ring
  B.pers += 3 * block_bytes((int64_t)R * kDotBlocks, 8) + block_bytes((int64_t)R * std::max<int64_t>(n_pq, 1), 8) +
            2 * block_bytes(R, sizeof(CgState)) + block_bytes((int64_t)R * kHistRing, 8);
  // work vectors
  const int64_t nu = n_obs * ns + n_tunk;
  B.work = 2 * block_bytes(y_bytes(fp64, R, n), 1) + 7 * block_bytes((int64_t)R * nu, 8);
  if (!fp64)
    B.work += block_bytes((int64_t)R * std::max<int64_t>(n_obs * ns, 1), 4) + 2 * block_bytes((int64_t)R * nu, 8) +
              (d->n_templates > 0 ? block_bytes((int64_t)R * nu, 8) : 0);
  // noise gradient
  if (d->filter_params) {
    const int64_t N64 = int64_t(1) << logn64;
    B.call_temps = block_bytes(std::max<int64_t>(n, 1), 8) + block_bytes((int64_t)nf_filt * n_c, 8) +
                   block_bytes(3 * (int64_t)nf_filt * (N64 + 1), 8) + block_bytes(3 * (int64_t)std::max(d->n_intervals, 1), 8) +
                   block_bytes((int64_t)std::max(lags_scratch_bytes(n_c, lag_len, batch),
                                                 symbol_scratch_bytes(logn64, true, nf_filt)), 1);
  }
  return B;
}

// Build a plan in the workspace ws of ws_bytes (the caller's), or, with ws = NULL,
// in one block of the bound's size that the plan allocates and frees itself.
void build_plan(mm_plan_s* P, const mm_desc_t* d, const int32_t* d_pix, const float* d_w, void* ws,
                size_t ws_bytes, hipStream_t s) {
  const PlanBounds bounds = plan_bounds(d);
  if (d->n_samples > 0 && !d_pix) fail(MM_EINVAL, "d_pix is NULL");
  if (d->n_stokes == 3 && d->n_samples > 0 && !d_w) fail(MM_EINVAL, "d_w is NULL for polarised pointing");

  P->ns = d->n_stokes;
  P->n_pix = d->n_pix;
  P->n_t = d->n_samples;
  P->n_iv = d->n_intervals;
  P->n_filt = d->n_filters;
  P->n_c = d->n_c;
  P->precision = d->precision;
  P->precond = d->precond;
  P->R = d->n_rhs;
  P->nf_req = d->n_f;
  P->shape_req = d->fft_shape;
  P->f_samp = d->f_samp;
  P->w = d_w;
  P->iv_start.assign(d->iv_start, d->iv_start + d->n_intervals + 1);
  P->iv_filter.assign(d->iv_filter, d->iv_filter + d->n_intervals);
  P->lag_len = d->lag_dft_len ? d->lag_dft_len : (1 << 20);
  if (d->filter_params) P->params.assign(d->filter_params, d->filter_params + 3 * (size_t)P->n_filt);

  const size_t need = bounds.total();
  if (ws) {
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) fail(MM_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
      fail(MM_EINVAL, "workspace of " + std::to_string(ws_bytes) + " bytes is below the " + std::to_string(need) +
                          " bytes mm_plan_workspace_size gives for this descriptor");
    P->ws = static_cast<char*>(ws);
    P->ws_size = ws_bytes;
  } else {
    hipchk(hipMalloc((void**)&P->ws, need), "hipMalloc of the plan's device memory");
    P->ws_owned = true;
    P->ws_size = need;
  }
  P->pers_lim = bounds.pers;
  P->work_top = P->tmp_base = P->tmp_peak = P->pers_lim;

  hipchk(hipGetDevice(&P->device), "hipGetDevice");
  P->own = stream_take(P->device);
  hipchk(hipEventCreateWithFlags(&P->ev_in, hipEventDisableTiming), "event");
  hipchk(hipEventCreateWithFlags(&P->ev_out, hipEventDisableTiming), "event");
  // one pinned block: the CG states, scalar slots, and the dot partials of dots2
  // (device-to-host copies into pageable memory are staged and serialise)
  const size_t st_bytes = (sizeof(CgState) * P->R + 255) & ~(size_t)255;
  const size_t pin_bytes = st_bytes + kPinSlots * 8 + sizeof(double) * 2 * P->R * kDotBlocks;
  hipchk(hipHostMalloc((void**)&P->st_host, pin_bytes, hipHostMallocDefault), "pinned state");
  P->pin = reinterpret_cast<char*>(P->st_host) + st_bytes;
  hipchk(hipHostMalloc((void**)&P->hist_host, sizeof(double) * P->R * kHistRing, hipHostMallocDefault),
         "pinned history");

  const int64_t n = P->n_t;
  // ---- pointing: range check, sort by pixel, observed layout
  build_layout(P, d_pix, P->n_pix, P->ns, d_w, P->px, s, "pointing index outside [-1, n_pix)");
  P->n_obs = P->px.n_obs;
  P->n_valid = P->px.n_valid;
  build_gather_order(P, s);
  setup_templates(P, d, s);

  // ---- noise filters
  P->lags = P->alloc<double>((int64_t)P->n_filt * P->n_c);
  if (d->filter_lags) {
    hipchk(hipMemcpyAsync(P->lags, d->filter_lags, sizeof(double) * P->n_filt * P->n_c,
                          hipMemcpyHostToDevice, s),
           "lag upload");
  } else {
    double* dparams = P->alloc<double>(3 * (int64_t)P->n_filt);
    P->d_params = dparams;
    hipchk(hipMemcpyAsync(dparams, P->params.data(), sizeof(double) * 3 * P->n_filt,
                          hipMemcpyHostToDevice, s),
           "parameter upload");
    const int batch = std::max(1, std::min(P->n_filt, 16));
    const size_t sb = lags_scratch_bytes(P->n_c, P->lag_len, batch);
    char* scr = P->temp<char>((int64_t)sb);
    hipchk(launch_lags(dparams, P->n_filt, P->f_samp, P->n_c, P->lag_len, P->lags, scr, sb, s),
           "lag construction");
    P->release(scr);
  }
  build_filter(P, P->fs_main, P->main_fp64(), s);
  // mixed plans: the float64 filter of the right-hand side and the residual replacements
  if (!P->main_fp64()) build_filter(P, P->fs64, true, s, true);

  // ---- preconditioner
  P->d_iv_start = P->alloc<int64_t>(P->n_iv + 1);
  P->d_iv_filter = P->alloc<int32_t>(P->n_iv);
  hipchk(hipMemcpyAsync(P->d_iv_start, P->iv_start.data(), 8 * (P->n_iv + 1), hipMemcpyHostToDevice, s), "copy");
  hipchk(hipMemcpyAsync(P->d_iv_filter, P->iv_filter.data(), 4 * P->n_iv, hipMemcpyHostToDevice, s), "copy");
  build_interval_hint(P, s);
  const int nm = P->ns == 1 ? 1 : 6;
  P->minv = P->alloc<double>(P->n_obs * nm);
  {
    int32_t* sing = P->temp<int32_t>(P->n_obs);
    unsigned long long* cnt = P->temp<unsigned long long>(1);
    hipchk(launch_precond_build(P->ns, P->precond, P->px.group, P->px.ptr, P->px.perm, P->px.w_pm, P->d_iv_start,
                                P->n_iv, P->d_iv_hint, P->iv_hint_shift, P->d_iv_filter, P->lags, P->n_c, P->n_obs,
                                P->minv, sing, s),
           "preconditioner");
    hipchk(launch_count_nonzero(sing, P->n_obs, cnt, s), "singular count");
    // read when first needed (plan info, end of a solve), not here: no wait in the plan build
    hipchk(hipMemcpyAsync(P->slot<unsigned long long>(kPinSingular), cnt, 8, hipMemcpyDeviceToHost, s), "copy");
    hipchk(hipEventCreateWithFlags(&P->ev_singular, hipEventDisableTiming), "event");
    hipchk(hipEventRecord(P->ev_singular, s), "event");
    P->release(sing);
    P->release(cnt);
  }
  build_template_precond(P, s);

  // ---- scatter layouts: the pixel-major arrays as they are, or a sliced copy that replaces them
  build_sell(P, P->px, P->ns, s);
  for (Template& T : P->tmpl)
    if (T.kind == MM_TMPL_ONEHOT) build_sell(P, T.lay, 1, s);

  // ---- p.q partial sums: the sky scatter's blocks, then each template's
  // (a scatter with no observed column writes none)
  P->n_pq = P->n_obs > 0 ? scatter_blocks(P->n_obs, P->px.sell.wps) : 0;
  for (Template& T : P->tmpl) {
    T.pq_slot = P->n_pq;
    T.pq_n = T.kind == MM_TMPL_ONEHOT ? (T.lay.n_obs > 0 ? scatter_blocks(T.lay.n_obs, T.lay.sell.wps) : 0) : 1;
    P->n_pq += T.pq_n;
  }

  // ---- white noise: N^-1 = f_b(0) on tiles of the intervals, no transforms
  if (P->n_c == 1) {
    std::vector<SampleTile> wt;
    for (int b = 0; b < P->n_iv; ++b)
      for (int64_t t0 = P->iv_start[b]; t0 < P->iv_start[b + 1]; t0 += kTileSamples)
        wt.push_back(SampleTile{t0, std::min<int64_t>(t0 + kTileSamples, P->iv_start[b + 1]), b, 0});
    if (wt.size() > (size_t)0x7fffffff) fail(MM_EUNSUPPORTED, "too many interval tiles");
    P->n_white_tiles = (int)wt.size();
    P->white_tiles = P->alloc<SampleTile>((int64_t)wt.size());
    if (!wt.empty())
      hipchk(hipMemcpyAsync(P->white_tiles, wt.data(), wt.size() * sizeof(SampleTile), hipMemcpyHostToDevice, s),
             "tile upload");
    hipchk(hipStreamSynchronize(s), "tiles");
  }

  // ---- work vectors: the build's temporaries are all released, the region is free
  if (!P->tmps.empty()) fail(MM_EDEVICE, "internal: plan temporaries outlive the build");
  P->part1 = P->alloc<double>((int64_t)P->R * kDotBlocks);
  P->part2 = P->alloc<double>((int64_t)P->R * kDotBlocks);
  P->part3 = P->alloc<double>((int64_t)P->R * kDotBlocks);
  P->part_pq = P->alloc<double>((int64_t)P->R * std::max(P->n_pq, 1));
  P->st = P->alloc<CgState>(P->R);
  P->st_prev = P->alloc<CgState>(P->R);
  P->hist = P->alloc<double>((int64_t)P->R * kHistRing);
  const int64_t ybytes = y_bytes(P->main_fp64(), P->R, n);
  P->y1 = P->work<char>(ybytes);
  P->y2 = P->work<char>(ybytes);
  const int64_t vn = (int64_t)P->R * P->nu();
  P->vx = P->work<double>(vn);
  P->vp = P->work<double>(vn);
  P->vr = P->work<double>(vn);
  P->vz = P->work<double>(vn);
  P->vq = P->work<double>(vn);
  P->vxb = P->work<double>(vn);
  P->vb = P->work<double>(vn);
  if (!P->main_fp64()) {
    // mixed iterations gather the search direction from a float32 copy of its map part
    // (half the map bytes; the gathered TOD is float32 anyway); reliable updates keep b
    // and the best iterate in float64, and the float64 residual passes reuse the TOD
    // work buffers, sized for one float64 row
    P->vp32 = P->work<float>((int64_t)P->R * std::max<int64_t>(P->vs32(), 1));
    P->vb64 = P->work<double>(vn);
    P->vxbest = P->work<double>(vn);
    if (!P->tmpl.empty()) P->vxacc = P->work<double>(vn);
    P->y64a = (double*)P->y1;
    P->y64b = (double*)P->y2;
  }
  // later temporaries (noise gradient) are stacked above the work vectors
  P->tmp_base = P->work_top;
  hipchk(hipEventCreateWithFlags(&P->ev_ready, hipEventDisableTiming), "event");
  hipchk(hipEventRecord(P->ev_ready, s), "event");
}

// queue one PCG iteration for every RHS
void enqueue_iteration(mm_plan_s* P, hipStream_t s) {
  const int R = P->R;
  // q = H p, with the partial sums of p.q formed by the scatters
  // (RHS that stopped iterating skip the TOD work: convergence is checked by
  // the host only every check_every iterations)
  gather_all(P, P->fs_main.fp64, P->vp, P->y1, R, s, P->st, P->vp32);
  weight(P, P->fs_main, P->y1, P->fs_main.fp64, P->y2, R, s, P->st);
  // the mixed-precision iteration without templates keeps q, z and p in float32 (q and z
  // in the first half of their float64 buffers, p in vp32): q is a float32 operator's
  // output, z only builds the next direction, and p is the direction the operator is
  // applied to, which x also moves along (x, r and the dots stay float64)
  const bool v32 = P->iter_f32();
  if (v32)
    hipchk(launch_scatter_q32(P->ns, P->px.sell, (const float*)P->y2, (float*)P->vq, P->nu(), P->n_obs, P->n_t, R,
                              s, P->vp32, P->vs32(), P->part_pq, P->n_pq, 0, P->st),
           "scatter");
  else
    scatter_all(P, P->fs_main.fp64, P->y2, P->vq, R, s, P->vp, P->st);
  hipchk(launch_cg_update(P->ns, P->vr, P->vq, P->vz, v32, P->minv, P->st, P->st_prev, P->n_obs,
                          P->nu(), P->minv_t, P->n_tunk, R, P->part_pq, P->n_pq, P->part2, P->part3, s),
         "update");
  if (v32 && P->x_inc32)
    hipchk(launch_cg_step_next(P->vdx32(), true, nullptr, P->vp32, true, P->vz, true, P->st, P->st_prev, P->part2,
                               P->part3, P->hist, kHistRing, P->nu(), R, s),
           "scalar step and next direction");
  else if (v32)
    hipchk(launch_cg_step_next(P->vx, false, P->vxb, P->vp32, true, P->vz, true, P->st, P->st_prev, P->part2,
                               P->part3, P->hist, kHistRing, P->nu(), R, s),
           "scalar step and next direction");
  else
    hipchk(launch_cg_step_next(P->vx, false, P->vxb, P->vp, false, P->vz, false, P->st, P->st_prev, P->part2,
                               P->part3, P->hist, kHistRing, P->nu(), R, s, P->vp32, P->nmap(), P->vs32()),
           "scalar step and next direction");
}

// per-RHS sums of x.y over [R][nu] vectors (float64, fixed order)
std::vector<double> dots(mm_plan_s* P, const double* x, const double* y, int R, hipStream_t s) {
  const int64_t nu = P->nu();
  std::vector<double> out(R, 0.0);
  const double* h = P->pin_dots();
  hipchk(launch_dot(x, y, nu, R, P->part1, s), "dot");
  hipchk(hipMemcpyAsync(P->pin_dots(), P->part1, sizeof(double) * R * kDotBlocks, hipMemcpyDeviceToHost, s), "copy");
  hipchk(hipStreamSynchronize(s), "dot");
  for (int r = 0; r < R; ++r)
    for (int i = 0; i < kDotBlocks; ++i) out[r] += h[(size_t)r * kDotBlocks + i];
  return out;
}

// per-RHS x.y and x.z with one host round trip
void dots2(mm_plan_s* P, const double* x, const double* y, const double* z, int R, hipStream_t s,
           std::vector<double>& xy, std::vector<double>& xz) {
  const int64_t nu = P->nu();
  double* h = P->pin_dots();
  hipchk(launch_dot(x, y, nu, R, P->part1, s), "dot");
  hipchk(launch_dot(x, z, nu, R, P->part2, s), "dot");
  hipchk(hipMemcpyAsync(h, P->part1, sizeof(double) * R * kDotBlocks, hipMemcpyDeviceToHost, s), "copy");
  hipchk(hipMemcpyAsync(h + (size_t)R * kDotBlocks, P->part2, sizeof(double) * R * kDotBlocks,
                        hipMemcpyDeviceToHost, s),
         "copy");
  hipchk(hipStreamSynchronize(s), "dot");
  xy.assign(R, 0.0);
  xz.assign(R, 0.0);
  for (int r = 0; r < R; ++r)
    for (int i = 0; i < kDotBlocks; ++i) {
      xy[r] += h[(size_t)r * kDotBlocks + i];
      xz[r] += h[(size_t)(R + r) * kDotBlocks + i];
    }
}

// queue `step` PCG iterations; a full block of k iterations runs as one hipGraph,
// captured once per plan (and k) from the plan's second solve on: a plan solved
// once gains nothing from the capture, and at the sizes where launches cost more
// than the kernels the capture is paid back by the second solve
void iterate_block(mm_plan_s* P, hipStream_t s, int step, int k, bool use_graph) {
  if (use_graph && step == k && k > 0 && P->solves > 0) {
    const int m = P->x_inc32 ? 1 : 0;
    if (!P->graph[m] || P->graph_k[m] != k) {
      if (P->graph[m]) {
        hipchk(hipGraphExecDestroy(P->graph[m]), "graph destroy");
        P->graph[m] = nullptr;
      }
      hipGraph_t g = nullptr;
      hipchk(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
      try {
        for (int i = 0; i < k; ++i) enqueue_iteration(P, s);
      } catch (...) {
        (void)hipStreamEndCapture(s, &g);   // unwinding: the first error is the one reported
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      hipchk(hipStreamEndCapture(s, &g), "end capture");
      hipchk(hipGraphInstantiate(&P->graph[m], g, nullptr, nullptr, 0), "graph instantiate");
      hipchk(hipGraphDestroy(g), "graph destroy");
      P->graph_k[m] = k;
    }
    hipchk(hipGraphLaunch(P->graph[m], s), "graph launch");
  } else {
    for (int i = 0; i < step; ++i) enqueue_iteration(P, s);
  }
}

// Iterations in the next block between host checks: a full block of k, or fewer when
// every active RHS is predicted to reach tol sooner from its residual rate since the
// previous check (a shorter block saves the launches past convergence; the estimate is
// padded, since a block that ends short costs another check).  For the mixed solver
// (ref_rel = each RHS's float64 residual at its last replacement) a block may run up
// to k_long iterations once the rate is known, but only as long as the residual is
// predicted to stay within max_drop decades of ref_rel: the float32 recurrence
// residual is trusted that far below the last float64 one, and fewer, longer blocks
// mean fewer float64 replacements.  Until the rate is known such a block is at most
// kMixedFirstBlock iterations.
struct BlockSizer {
  std::vector<double> rel;
  std::vector<int> iter;
  explicit BlockSizer(int R) : rel(R, 0.0), iter(R, -1) {}
  int next(const CgState* st, int k, double tol, int k_long = 0, double max_drop = 0.0,
           const double* ref_rel = nullptr) {
    int need = 0, cap = std::max(k, k_long);
    bool any = false, all_rates = true;
    for (size_t r = 0; r < rel.size(); ++r) {
      const CgState& c = st[r];
      if (!c.active) continue;
      any = true;
      int est = k;
      if (iter[r] >= 0 && c.iter > iter[r] && rel[r] > c.rel && c.rel > 0) {
        const double rate = std::log(c.rel / rel[r]) / (double)(c.iter - iter[r]);   // per iteration, < 0
        if (tol > 0 && c.rel > tol) est = (int)std::ceil(1.25 * std::log(tol / c.rel) / rate) + 1;
        if (max_drop > 0 && ref_rel) {
          const double left = max_drop * std::log(10.0) - std::log(std::max(ref_rel[r], c.rel) / c.rel);
          cap = std::min(cap, std::max(1, (int)(left / -rate)));
        }
      } else {
        all_rates = false;
      }
      need = std::max(need, est);
      rel[r] = c.rel;
      iter[r] = c.iter;
    }
    // without a rate (first block, or a residual that rose) a mixed block is at most
    // kMixedFirstBlock iterations, whatever check_every asks
    const int longest = (max_drop > 0 && ref_rel) ? (all_rates ? cap : std::min(k, kMixedFirstBlock)) : k;
    return any ? std::max(1, std::min(longest, need)) : k;
  }
};

// Copy the device's residual ring after a block and append the iterations the host
// has not seen yet to hseq [R][n_max + 1] (blocks are shorter than the ring).
void read_history(mm_plan_s* P, int n_max, std::vector<int>& seen, std::vector<double>& hseq, double scale = 1.0,
                  const std::vector<int>* offset = nullptr) {
  for (int r = 0; r < P->R; ++r) {
    const CgState& c = P->st_host[r];
    const int base = offset ? (*offset)[r] : 0;
    for (int i = seen[r] + 1; i <= c.iter; ++i)
      if (base + i <= n_max)
        hseq[(size_t)r * (n_max + 1) + base + i] = scale * P->hist_host[(size_t)r * kHistRing + i % kHistRing];
    seen[r] = std::max(seen[r], c.iter);
  }
}

// PCG on H x = vb (observed layout) in the iteration precision of fs_main.
// vb must hold the right-hand sides; x0 is read from vx when have_x0.  On
// exit vxb holds the lowest-residual iterate (vx is then undefined) and st_host
// the final states;
// hseq [R][n_max + 1] the relative residual per iteration (entry 0 = start).
void run_pcg(mm_plan_s* P, hipStream_t s, double tol, int n_max, bool fixed, int check_every,
             bool use_graph, bool have_x0, std::vector<double>& hseq) {
  const int R = P->R;
  const int64_t nu = P->nu();
  if (have_x0) {
    apply_H_obs(P, P->fs_main, P->vx, P->vq, P->y1, P->y2, R, s);
    hipchk(launch_sub(P->vr, P->vb, P->vq, (int64_t)R * nu, s), "residual");
  } else {
    hipchk(launch_fill_f64(P->vx, 0.0, (int64_t)R * nu, s), "fill");
    hipchk(hipMemcpyAsync(P->vr, P->vb, sizeof(double) * R * nu, hipMemcpyDeviceToDevice, s), "copy");
  }
  hipchk(launch_apply_precond(P->ns, P->minv, P->vr, P->vz, P->n_obs, nu, P->minv_t, P->n_tunk, R, s),
         "precondition");
  hipchk(hipMemcpyAsync(P->vp, P->vz, sizeof(double) * R * nu, hipMemcpyDeviceToDevice, s), "copy");
  sync_p32(P, s);
  hipchk(launch_dot(P->vb, P->vb, nu, R, P->part1, s), "dot");
  hipchk(launch_dot(P->vr, P->vr, nu, R, P->part2, s), "dot");
  hipchk(launch_dot(P->vr, P->vz, nu, R, P->part3, s), "dot");
  hipchk(launch_cg_init(P->st, P->part1, P->part2, P->part3, tol, fixed ? 1 : 0, R, P->hist, kHistRing, s),
         "init");

  hseq.assign((size_t)R * (n_max + 1), std::nan(""));
  std::vector<int> seen(R, -1);
  auto all_done = [&]() {
    hipchk(hipMemcpyAsync(P->st_host, P->st, sizeof(CgState) * R, hipMemcpyDeviceToHost, s), "state copy");
    hipchk(hipMemcpyAsync(P->hist_host, P->hist, sizeof(double) * R * kHistRing, hipMemcpyDeviceToHost, s),
           "history copy");
    hipchk(hipStreamSynchronize(s), "solve");
    read_history(P, n_max, seen, hseq);
    for (int r = 0; r < R; ++r)
      if (P->st_host[r].active) return false;
    return true;
  };

  int done = 0;
  bool finished = all_done();
  const int k = std::min({check_every, std::max(1, n_max), kMaxCheckEvery});
  BlockSizer sizer(R);
  while (!finished && done < n_max) {
    const int step = std::min(fixed ? k : sizer.next(P->st_host, k, tol), n_max - done);
    iterate_block(P, s, step, k, use_graph);
    done += step;
    finished = all_done();
  }
  // the iterations keep each RHS's lowest-residual iterate in vx or vxb (CgState.xbest):
  // gather them in vxb
  for (int r = 0; r < R; ++r)
    if (P->st_host[r].xbest == 0)
      hipchk(hipMemcpyAsync(P->vxb + (int64_t)r * nu, P->vx + (int64_t)r * nu, sizeof(double) * nu,
                            hipMemcpyDeviceToDevice, s), "copy");
}

// Float64 TOD rows one float64 pass can take at once: the TOD work buffers hold R rows
// of the plan's own precision, so R / 2 float64 rows in a mixed plan
int rows64(const mm_plan_s* P) { return P->main_fp64() ? P->R : std::max(1, P->R / 2); }

// out_r = b64_r - H64 x_r for the RHS r0 .. r0 + nr - 1, in float64 (through the float64
// filter), rows64 of them per pass so that the pointing is read once per group
void residual64_rows(mm_plan_s* P, const double* x, double* out, int r0, int nr, hipStream_t s) {
  const int64_t nu = P->nu();
  const FilterSetup& f64 = P->main_fp64() ? P->fs_main : P->fs64;
  void* ya = P->main_fp64() ? P->y1 : (void*)P->y64a;
  void* yb = P->main_fp64() ? P->y2 : (void*)P->y64b;
  const int B = rows64(P);
  for (int a = r0; a < r0 + nr; a += B) {
    const int k = std::min(B, r0 + nr - a);
    apply_H_obs(P, f64, x + (int64_t)a * nu, P->vq, ya, yb, k, s);
    hipchk(launch_sub(out + (int64_t)a * nu, P->vb64 + (int64_t)a * nu, P->vq, (int64_t)k * nu, s), "residual");
  }
}

// the same for the RHS listed in rows (ascending), consecutive ones together
void residual64_list(mm_plan_s* P, const double* x, double* out, const std::vector<int>& rows, hipStream_t s) {
  for (size_t i = 0; i < rows.size();) {
    size_t j = i + 1;
    while (j < rows.size() && rows[j] == rows[j - 1] + 1) ++j;
    residual64_rows(P, x, out, rows[i], (int)(j - i), s);
    i = j;
  }
}

// Right-hand side of a solve: b = P^T N^-1 d from a TOD, or a map given directly.
struct RhsSource {
  const void* tod = nullptr;
  bool tod64 = false;
  const double* map = nullptr;   // global layout [R][n_pix][ns]
};

// b64 of every RHS through the float64 filter, rows64 per pass
void make_rhs64(mm_plan_s* P, const RhsSource& src, hipStream_t s);

// b (observed layout) of RHS rows [r0, r0 + nr) with the filter fs into dst
void make_rhs(mm_plan_s* P, const RhsSource& src, const FilterSetup& fs, int r0, int nr, double* dst,
              void* yb, hipStream_t s) {
  if (src.map) {
    to_obs(P, src.map + (int64_t)r0 * P->ng(), dst, nr, s);
  } else {
    const int esz = src.tod64 ? 8 : 4;
    rhs_obs(P, fs, (const char*)src.tod + (size_t)r0 * P->n_t * esz, src.tod64, dst, yb, nr, s);
  }
}

void make_rhs64(mm_plan_s* P, const RhsSource& src, hipStream_t s) {
  const int64_t nu = P->nu();
  const int B = rows64(P);
  for (int a = 0; a < P->R; a += B) {
    const int k = std::min(B, P->R - a);
    make_rhs(P, src, P->fs64, a, k, P->vb64 + (int64_t)a * nu, P->y64b, s);
  }
}

void solve_impl(mm_plan_s* P, const RhsSource& src, double* d_x, const mm_solve_opts_t* o_in,
                mm_solve_info_t* info, hipStream_t caller, mm_status_t* result) {
  mm_solve_opts_t o;
  mm_solve_opts_default(&o);
  if (o_in) o = *o_in;
  if (!d_x) fail(MM_EINVAL, "d_x is NULL");
  if (!src.map && !src.tod && P->n_t > 0) fail(MM_EINVAL, "right-hand side is NULL");
  if (o.fixed_iters < 0 || o.max_iter < 0) fail(MM_EINVAL, "iteration counts must be >= 0");
  if (!(o.tol >= 0)) fail(MM_EINVAL, "tol must be >= 0");
  if (o.check_every < 1) o.check_every = 1;
  const bool fixed = o.fixed_iters > 0;
  const int n_max = fixed ? o.fixed_iters : o.max_iter;
  const int R = P->R;
  const int64_t nu = P->nu();
  const bool refine = !P->main_fp64() && o.refine && !fixed;
  hipStream_t s = P->own;

  // order the plan stream after the plan's build and the caller's work
  wait_ready(P, s);
  hipchk(hipEventRecord(P->ev_in, caller), "event");
  hipchk(hipStreamWaitEvent(s, P->ev_in, 0), "event wait");

  std::vector<int> iters(R, 0), best_iter(R, 0);
  std::vector<double> best_rel(R, 0.0), tres(R, std::nan(""));
  std::vector<double> hist_out((size_t)R * (n_max + 1), std::nan(""));
  bool notconv = false;

  if (!refine) {
    make_rhs(P, src, P->fs_main, 0, R, P->vb, P->y2, s);
    if (o.d_x0) to_obs(P, o.d_x0, P->vx, R, s);
    run_pcg(P, s, o.tol, n_max, fixed, o.check_every, o.use_graph != 0, o.d_x0 != nullptr, hist_out);
    for (int r = 0; r < R; ++r) {
      const CgState& c = P->st_host[r];
      iters[r] = c.iter;
      best_iter[r] = c.best_iter;
      best_rel[r] = c.best_rel;
      if (!fixed && c.bnorm > 0 && !(c.rel <= o.tol) && !(c.best_rel <= o.tol)) notconv = true;
    }
    to_glob(P, P->vxb, d_x, R, s);
  } else if (P->tmpl.empty()) {
    // Mixed precision with reliable updates (float64 residual replacement): H is
    // applied in float32, r, b and the dots are float64, and in the float32 iteration
    // (no templates) q, z and p are float32 and, late in the solve, x moves by a float32
    // increment folded into the float64 x at each replacement.  At the host's check
    // points, for each RHS whose recurrence residual fell a thousandfold since its last
    // replacement (or reached tol, or stopped), the residual is replaced by the float64
    // true residual b - H64 x, z = M r and rho = r.z are recomputed, and CG continues
    // along the same direction p (no restart).  Blocks between checks are sized
    // (BlockSizer) so that the recurrence residual is not predicted to fall more than
    // kMixedMaxDrop decades below the last float64 one.  The iterate with the lowest true
    // residual is returned.
    make_rhs64(P, src, s);
    hipchk(hipMemcpyAsync(P->vb, P->vb64, sizeof(double) * R * nu, hipMemcpyDeviceToDevice, s), "copy");
    if (o.d_x0) {
      to_obs(P, o.d_x0, P->vx, R, s);
      residual64_rows(P, P->vx, P->vr, 0, R, s);
    } else {
      hipchk(launch_fill_f64(P->vx, 0.0, (int64_t)R * nu, s), "fill");
      hipchk(hipMemcpyAsync(P->vr, P->vb, sizeof(double) * R * nu, hipMemcpyDeviceToDevice, s), "copy");
    }
    hipchk(hipMemcpyAsync(P->vxbest, P->vx, sizeof(double) * R * nu, hipMemcpyDeviceToDevice, s), "copy");
    hipchk(launch_apply_precond(P->ns, P->minv, P->vr, P->vz, P->n_obs, nu, P->minv_t, P->n_tunk, R, s),
           "precondition");
    hipchk(hipMemcpyAsync(P->vp, P->vz, sizeof(double) * R * nu, hipMemcpyDeviceToDevice, s), "copy");
    sync_p32(P, s);
    // Once every RHS's float64 residual is below kIncrementFrom, float32 iterations move
    // x by a float32 increment (half the bytes of the float64 read and write), folded
    // into the float64 x for the RHS of each replacement.
    struct IncrementMode {
      mm_plan_s* P;
      ~IncrementMode() { P->x_inc32 = false; }
    } increment_mode{P};
    hipchk(launch_dot(P->vb, P->vb, nu, R, P->part1, s), "dot");
    hipchk(launch_dot(P->vr, P->vr, nu, R, P->part2, s), "dot");
    hipchk(launch_dot(P->vr, P->vz, nu, R, P->part3, s), "dot");
    hipchk(launch_cg_init(P->st, P->part1, P->part2, P->part3, o.tol, 0, R, P->hist, kHistRing, s), "init");
    hipchk(hipMemcpyAsync(P->st_host, P->st, sizeof(CgState) * R, hipMemcpyDeviceToHost, s), "state copy");
    hipchk(hipStreamSynchronize(s), "init");
    std::vector<double> last_true(R), best_true(R);
    std::vector<int> rep_iter(R, 0);
    for (int r = 0; r < R; ++r) {
      CgState& c = P->st_host[r];
      last_true[r] = best_true[r] = c.rel;
      best_rel[r] = c.rel;
      hist_out[(size_t)r * (n_max + 1)] = c.rel;
      c.best_rel = -1.0;            // the device keeps no best copy: the host tracks true residuals
      c.xbest = -1;                 // and x stays in vx (replacements read it there)
    }
    hipchk(hipMemcpyAsync(P->st, P->st_host, sizeof(CgState) * R, hipMemcpyHostToDevice, s), "state copy");

    // replace the residual of the RHS in `rows` (and restart the direction p = z of
    // those that broke down); returns after updating the device states
    std::vector<int> restarted(R, -1);
    auto replace = [&](const std::vector<int>& rows) {
      if (P->x_inc32)
        for (int r : rows)
          hipchk(launch_fold_f32(P->vx + (int64_t)r * nu, P->vdx32() + (int64_t)r * nu, nu, s), "fold");
      residual64_list(P, P->vx, P->vr, rows, s);
      hipchk(launch_apply_precond(P->ns, P->minv, P->vr, P->vz, P->n_obs, nu, P->minv_t, P->n_tunk, R, s),
             "precondition");
      for (int r : rows)
        if (P->st_host[r].breakdown) {
          hipchk(hipMemcpyAsync(P->vp + (int64_t)r * nu, P->vz + (int64_t)r * nu, sizeof(double) * nu,
                                hipMemcpyDeviceToDevice, s), "restart");
          if (P->vp32)   // the iteration's direction (the only one in a float32 iteration)
            hipchk(launch_rows_to_f32(P->vz + (int64_t)r * nu, nu, P->vp32 + (int64_t)r * P->vs32(), P->vs32(),
                                      P->nmap(), 1, s), "restart");
        }
      std::vector<double> rr, rz;
      dots2(P, P->vr, P->vr, P->vz, R, s, rr, rz);
      for (int r : rows) {
        CgState& c = P->st_host[r];
        const double tr = c.bnorm > 0 ? std::sqrt(rr[r]) / c.bnorm : 0.0;
        last_true[r] = tr;
        rep_iter[r] = c.iter;
        if (c.iter <= n_max) hist_out[(size_t)r * (n_max + 1) + c.iter] = tr;
        if (tr < best_true[r]) {
          best_true[r] = tr;
          best_iter[r] = c.iter;
          hipchk(hipMemcpyAsync(P->vxbest + (int64_t)r * nu, P->vx + (int64_t)r * nu, sizeof(double) * nu,
                                hipMemcpyDeviceToDevice, s), "copy");
        }
        // p.q <= 0 can occur where the float32 operator is indefinite (directions
        // the float64 H nearly annihilates): restart once per iteration count
        bool give_up = false;
        if (c.breakdown) {
          give_up = restarted[r] == c.iter;
          restarted[r] = c.iter;
        }
        c.rho = rz[r];
        c.rel = tr;
        c.breakdown = 0;
        c.copy_best = 0;
        c.active = (c.bnorm > 0 && tr > o.tol && c.iter < n_max && !give_up) ? 1 : 0;
      }
      hipchk(hipMemcpyAsync(P->st, P->st_host, sizeof(CgState) * R, hipMemcpyHostToDevice, s), "state copy");
    };

    std::vector<int> seen(R, 0);   // iterations whose residual the host has read
    const int k = std::min({std::max(o.check_every, 1), std::max(1, n_max), kMaxCheckEvery});
    int done = 0;
    auto any_active = [&]() {
      for (int r = 0; r < R; ++r)
        if (P->st_host[r].active) return true;
      return false;
    };
    BlockSizer sizer(R);
    while (any_active() && done < n_max) {
      const int step = std::min(sizer.next(P->st_host, k, o.tol, 2 * k, kMixedMaxDrop, last_true.data()), n_max - done);
      iterate_block(P, s, step, k, o.use_graph != 0);
      done += step;
      hipchk(hipMemcpyAsync(P->st_host, P->st, sizeof(CgState) * R, hipMemcpyDeviceToHost, s), "state copy");
      hipchk(hipMemcpyAsync(P->hist_host, P->hist, sizeof(double) * R * kHistRing, hipMemcpyDeviceToHost, s),
             "history copy");
      hipchk(hipStreamSynchronize(s), "solve");
      read_history(P, n_max, seen, hist_out);
      std::vector<int> rows;
      for (int r = 0; r < R; ++r) {
        const CgState& c = P->st_host[r];
        if (c.bnorm > 0 && (c.iter > rep_iter[r] || (c.breakdown && restarted[r] != c.iter)) &&
            (!c.active || c.rel <= o.tol || c.rel <= kMixedReplaceFall * last_true[r] || done >= n_max))
          rows.push_back(r);
      }
      if (!rows.empty()) replace(rows);
      if (P->iter_f32() && !P->x_inc32) {
        bool all = true;
        for (int r = 0; r < R; ++r) {
          const CgState& c = P->st_host[r];
          all = all && (c.bnorm <= 0 || !c.active || (rep_iter[r] > 0 && last_true[r] <= kIncrementFrom));
        }
        if (all) {
          hipchk(launch_fill_i32(reinterpret_cast<int32_t*>(P->vdx32()), 0, (int64_t)R * nu, s), "fill");
          P->x_inc32 = true;
        }
      }
    }
    for (int r = 0; r < R; ++r) {
      const CgState& c = P->st_host[r];
      iters[r] = c.iter;
      best_rel[r] = best_true[r];
      tres[r] = best_true[r];
      if (c.bnorm > 0 && !(best_true[r] <= o.tol)) notconv = true;
    }
    to_glob(P, P->vxbest, d_x, R, s);
  } else {
    // Plans with templates, whose extended system can be singular or nearly so:
    // float64 residual correction by restarted solves.  The float32-operator PCG
    // solves H d = r64 for a correction from d = 0 to a bounded depth, the float64
    // operator recomputes the true residual r64 = b64 - H64 x, and the iterate with
    // the lowest true residual is kept.  (One long float32-operator CG, as in the
    // reliable updates, drifts along directions the float64 H nearly annihilates:
    // invisible in the residual, not in the fitted TOD.)
    double* const vr64 = P->vb;   // the true residual is the correction equation's right-hand side
    make_rhs64(P, src, s);
    if (o.d_x0) {
      to_obs(P, o.d_x0, P->vxacc, R, s);
      residual64_rows(P, P->vxacc, vr64, 0, R, s);
    } else {
      hipchk(launch_fill_f64(P->vxacc, 0.0, (int64_t)R * nu, s), "fill");
      hipchk(hipMemcpyAsync(vr64, P->vb64, sizeof(double) * R * nu, hipMemcpyDeviceToDevice, s), "copy");
    }
    hipchk(hipMemcpyAsync(P->vxbest, P->vxacc, sizeof(double) * R * nu, hipMemcpyDeviceToDevice, s), "copy");
    const std::vector<double> bb = dots(P, P->vb64, P->vb64, R, s);
    std::vector<double> rel(R), bn(R);
    {
      const std::vector<double> rr = dots(P, vr64, vr64, R, s);
      for (int r = 0; r < R; ++r) {
        bn[r] = std::sqrt(bb[r]);
        rel[r] = bn[r] > 0 ? std::sqrt(rr[r]) / bn[r] : 0.0;
        best_rel[r] = rel[r];
        hist_out[(size_t)r * (n_max + 1)] = rel[r];
      }
    }
    for (int outer = 0; outer < 30; ++outer) {
      // right-hand sides of the correction equation; RHS already converged get 0
      double worst = 0.0;
      bool any = false;
      for (int r = 0; r < R; ++r) {
        const bool act = bn[r] > 0 && rel[r] > o.tol && iters[r] < n_max;
        double* dst = P->vb + (int64_t)r * nu;       // = the residual r64 of RHS r
        if (act) {
          worst = std::max(worst, rel[r]);
          any = true;
        } else {
          hipchk(launch_fill_f64(dst, 0.0, nu, s), "fill");
        }
      }
      if (!any) break;
      // inner tolerance: reach the target in this pass if the float32 operator allows,
      // otherwise gain about five decades
      const double tau = std::max(o.tol / worst, 1e-5);
      int budget = 0;
      for (int r = 0; r < R; ++r) budget = std::max(budget, n_max - iters[r]);
      std::vector<double> inner;   // the correction solve's residuals, relative to its right-hand side
      run_pcg(P, s, tau, budget, false, o.check_every, o.use_graph != 0, false, inner);
      // x += d (rows of converged RHS add 0)
      hipchk(launch_axpby(P->vxacc, P->vxb, 1.0, 1.0, (int64_t)R * nu, s), "accumulate");
      residual64_rows(P, P->vxacc, vr64, 0, R, s);
      const std::vector<double> rr = dots(P, vr64, vr64, R, s);
      for (int r = 0; r < R; ++r) {
        const CgState& c = P->st_host[r];
        const double scale = rel[r];
        for (int i = 1; i <= c.iter && iters[r] + i <= n_max; ++i)
          hist_out[(size_t)r * (n_max + 1) + iters[r] + i] = scale * inner[(size_t)r * (budget + 1) + i];
        iters[r] += c.iter;
        rel[r] = bn[r] > 0 ? std::sqrt(rr[r]) / bn[r] : 0.0;
        if (iters[r] <= n_max) hist_out[(size_t)r * (n_max + 1) + iters[r]] = rel[r];
        if (rel[r] < best_rel[r]) {
          best_rel[r] = rel[r];
          best_iter[r] = iters[r];
          hipchk(hipMemcpyAsync(P->vxbest + (int64_t)r * nu, P->vxacc + (int64_t)r * nu, sizeof(double) * nu,
                                hipMemcpyDeviceToDevice, s), "copy");
        }
      }
    }
    for (int r = 0; r < R; ++r) {
      tres[r] = best_rel[r];
      if (bn[r] > 0 && !(best_rel[r] <= o.tol)) notconv = true;
    }
    to_glob(P, P->vxbest, d_x, R, s);
  }

  if (o.true_residual && P->n_obs > 0 && !refine) {
    // ||b - H x|| / ||b|| in float64, one RHS at a time
    const FilterSetup& f64 = P->main_fp64() ? P->fs_main : P->fs64;
    void* ya = P->main_fp64() ? P->y1 : (void*)P->y64a;
    void* yb = P->main_fp64() ? P->y2 : (void*)P->y64b;
    for (int r = 0; r < R; ++r) {
      make_rhs(P, src, f64, r, 1, P->vr, yb, s);                            // b (float64)
      apply_H_obs(P, f64, P->vxb + (int64_t)r * nu, P->vq, ya, yb, 1, s);   // H x
      hipchk(launch_sub(P->vz, P->vr, P->vq, nu, s), "residual");
      const double b2 = dots(P, P->vr, P->vr, 1, s)[0];
      const double r2 = dots(P, P->vz, P->vz, 1, s)[0];
      tres[r] = b2 > 0 ? std::sqrt(r2 / b2) : 0.0;
    }
  }

  std::vector<double> merr(R, std::nan(""));
  if (o.map_error && nu > 0) {
    // Distance of the returned map x to the exact float64 solution x* = H^-1 b: the
    // error e = x* - x solves H e = b - H x, with the residual formed in float64 and
    // the correction equation solved by PCG with the plan's operator to 1e-2 of its
    // right-hand side, which gives ||e|| to about two digits.  The float32 operator of
    // a mixed plan differs from H by far less than that.
    const double* xs = refine ? P->vxbest : P->vxb;
    const std::vector<double> xx = dots(P, xs, xs, R, s);
    if (P->main_fp64()) {
      for (int r = 0; r < R; ++r) {
        apply_H_obs(P, P->fs_main, xs + (int64_t)r * nu, P->vq, P->y1, P->y2, 1, s);
        hipchk(launch_sub(P->vr + (int64_t)r * nu, P->vb + (int64_t)r * nu, P->vq, nu, s), "residual");
      }
    } else {
      if (!refine)
        make_rhs64(P, src, s);
      residual64_rows(P, xs, P->vr, 0, R, s);
    }
    hipchk(hipMemcpyAsync(P->vb, P->vr, sizeof(double) * R * nu, hipMemcpyDeviceToDevice, s), "copy");
    std::vector<double> inner;
    run_pcg(P, s, 1e-2, 50, false, o.check_every, o.use_graph != 0, false, inner);
    const std::vector<double> ee = dots(P, P->vxb, P->vxb, R, s);
    for (int r = 0; r < R; ++r) merr[r] = xx[r] > 0 ? std::sqrt(ee[r] / xx[r]) : (ee[r] > 0 ? INFINITY : 0.0);
  }

  hipchk(hipStreamSynchronize(s), "solve end");
  hipchk(hipEventRecord(P->ev_out, s), "event");
  hipchk(hipStreamWaitEvent(caller, P->ev_out, 0), "event wait");

  if (info) {
    for (int r = 0; r < R; ++r) {
      if (info->iters) info->iters[r] = iters[r];
      if (info->best_iter) info->best_iter[r] = best_iter[r];
      if (info->best_rel_res) info->best_rel_res[r] = best_rel[r];
      if (info->true_rel_res) info->true_rel_res[r] = tres[r];
      if (info->map_error) info->map_error[r] = merr[r];
    }
    if (info->history) std::memcpy(info->history, hist_out.data(), sizeof(double) * hist_out.size());
  }
  if (singular_count(P) > 0) {
    g_last_error = std::to_string(P->n_singular) + " singular preconditioner block(s)";
    *result = MM_ESINGULAR;
  } else if (notconv) {
    g_last_error = "tolerance not reached within max_iter";
    *result = MM_ENOTCONV;
  }
}

}  // namespace

namespace {

// Arguments of the plan-free lag construction; returns its smallest scratch (one
// filter per batch).
size_t check_lag_args(const double* d_params, int32_t n_filters, double f_samp, int32_t n_c, int64_t lag_len,
                      int32_t deriv, const double* d_lags) {
  if (!d_params || !d_lags) fail(MM_EINVAL, "NULL argument");
  if (n_filters < 1) fail(MM_EINVAL, "n_filters must be >= 1");
  if (n_c < 1) fail(MM_EINVAL, "n_c must be >= 1");
  if (!(f_samp > 0) || !std::isfinite(f_samp)) fail(MM_EINVAL, "f_samp must be positive");
  if (deriv < 0 || deriv > 3) fail(MM_EINVAL, "deriv must be 0 (lags) or 1 .. 3 (d/dsigma, d/df_knee, d/dalpha)");
  const int ncp = 1 << std::max(kMinLogN, ilog2(n_c));
  if (ncp > (1 << ols_max_logn(true))) fail(MM_EUNSUPPORTED, "n_c too large for the lag construction");
  if (!is_pow2(lag_len) || lag_len < 4 * (int64_t)ncp || lag_len > (int64_t(1) << 30))
    fail(MM_EINVAL, "lag_dft_len must be a power of two in [4 n_c, 2^30]");
  return lags_scratch_bytes(n_c, lag_len, 1);
}

// The allocation-free lag construction's scratch: one array per device, taken by
// every mm_noise_lags_noalloc call on that device.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

// Device address of `scratch` on the current device, looked up once per device.
void* noalloc_scratch() {
  static std::mutex mu;
  static void* addr[64] = {};
  int dev = 0;
  hipchk(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) fail(MM_EUNSUPPORTED, "device id above 63");
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    hipchk(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
    addr[dev] = p;
  }
  return addr[dev];
}

}  // namespace

namespace {

mm_status_t plan_impl(const mm_desc_t* desc, const int32_t* d_pix, const float* d_w, void* ws, size_t ws_bytes,
                      void* stream, mm_plan_t* out_plan) {
  if (!out_plan) {
    g_last_error = "out_plan is NULL";
    return MM_EINVAL;
  }
  *out_plan = nullptr;
  mm_plan_s* P = nullptr;
  const mm_status_t st = guarded([&] {
    P = new mm_plan_s();
    build_plan(P, desc, d_pix, d_w, ws, ws_bytes, as_stream(stream));
  });
  if (st != MM_OK) {
    delete P;
    return st;
  }
  *out_plan = P;
  return MM_OK;
}

}  // namespace

extern "C" {

void mm_solve_opts_default(mm_solve_opts_t* o) {
  if (!o) return;
  o->tol = 1e-6;
  o->max_iter = 50;
  o->fixed_iters = 0;
  o->check_every = 8;
  o->use_graph = 1;
  o->true_residual = 0;
  o->d_x0 = nullptr;
  o->refine = 1;
  o->map_error = 0;
}


mm_status_t mm_plan_workspace_size(const mm_desc_t* desc, size_t* bytes) {
  return guarded([&] {
    if (!bytes) fail(MM_EINVAL, "bytes is NULL");
    *bytes = plan_bounds(desc).total();
  });
}

mm_status_t mm_plan(const mm_desc_t* desc, const int32_t* d_pix, const float* d_w, void* d_ws, size_t ws_bytes,
                    void* stream, mm_plan_t* out_plan) {
  if (!d_ws) {
    g_last_error = "d_ws is NULL";
    if (out_plan) *out_plan = nullptr;
    return MM_EINVAL;
  }
  return plan_impl(desc, d_pix, d_w, d_ws, ws_bytes, stream, out_plan);
}

mm_status_t mm_plan_create(const mm_desc_t* desc, const int32_t* d_pix, const float* d_w, void* stream,
                           mm_plan_t* out_plan) {
  return plan_impl(desc, d_pix, d_w, nullptr, 0, stream, out_plan);
}

mm_status_t mm_destroy(mm_plan_t plan) {
  return guarded([&] { delete plan; });
}

mm_status_t mm_plan_destroy(mm_plan_t plan) { return mm_destroy(plan); }

mm_status_t mm_plan_get_info(mm_plan_t P, mm_plan_info_t* info) {
  return guarded([&] {
    if (!P || !info) fail(MM_EINVAL, "NULL argument");
    info->n_obs = P->n_obs;
    info->n_valid = P->n_valid;
    info->n_f = P->fs_main.nf;
    info->n_chunks = P->fs_main.n_chunks;
    info->n_singular = singular_count(P);
    info->n_sliced = P->px.sell_entries;
    info->n_tmpl = P->n_tglob;
    info->fft_shape = P->fs_main.variant + 1;
    info->device_bytes = P->bytes();
  });
}

mm_status_t mm_hits(mm_plan_t P, int32_t* d_hits, void* stream) {
  return guarded([&] {
    if (!P || !d_hits) fail(MM_EINVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    wait_ready(P, s);
    hipchk(launch_hits(P->px.ptr, P->px.obs2glob, d_hits, P->n_obs, P->n_pix, s), "hits");
  });
}

mm_status_t mm_filter_lags(mm_plan_t P, double* lags_out, void* stream) {
  return guarded([&] {
    if (!P || !lags_out) fail(MM_EINVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    wait_ready(P, s);
    hipchk(hipMemcpyAsync(lags_out, P->lags, sizeof(double) * (size_t)P->n_filt * P->n_c, hipMemcpyDeviceToHost, s),
           "lag download");
    hipchk(hipStreamSynchronize(s), "lag download");
  });
}

mm_status_t mm_unpoint(mm_plan_t P, const double* d_x, void* d_y, int32_t tod_dtype, void* stream) {
  return guarded([&] {
    if (!P || !d_x || (!d_y && P->n_t > 0)) fail(MM_EINVAL, "NULL argument");
    check_tod_dtype(tod_dtype);
    hipStream_t s = as_stream(stream);
    wait_ready(P, s);
    to_obs(P, d_x, P->vq, P->R, s);
    gather_all(P, tod_dtype == MM_F64, P->vq, d_y, P->R, s);
  });
}

mm_status_t mm_point(mm_plan_t P, const void* d_y, int32_t tod_dtype, double* d_x, void* stream) {
  return guarded([&] {
    if (!P || !d_x || (!d_y && P->n_t > 0)) fail(MM_EINVAL, "NULL argument");
    check_tod_dtype(tod_dtype);
    hipStream_t s = as_stream(stream);
    wait_ready(P, s);
    scatter_all(P, tod_dtype == MM_F64, d_y, P->vq, P->R, s);
    to_glob(P, P->vq, d_x, P->R, s);
  });
}

mm_status_t mm_weight(mm_plan_t P, const void* d_y_in, void* d_y_out, int32_t tod_dtype, void* stream) {
  return guarded([&] {
    if (!P || ((!d_y_in || !d_y_out) && P->n_t > 0)) fail(MM_EINVAL, "NULL argument");
    check_tod_dtype(tod_dtype);
    if (d_y_in == d_y_out && P->n_t > 0) fail(MM_EINVAL, "y_out must not alias y_in");
    hipStream_t s = as_stream(stream);
    wait_ready(P, s);
    const bool in64 = tod_dtype == MM_F64;
    const bool t64 = P->main_fp64();
    if (in64 == t64) {
      weight(P, P->fs_main, d_y_in, in64, d_y_out, P->R, s);
    } else {
      weight(P, P->fs_main, d_y_in, in64, P->y2, P->R, s);
      hipchk(launch_convert(t64, in64, P->y2, d_y_out, (int64_t)P->R * P->n_t, s), "convert");
    }
  });
}

mm_status_t mm_apply_A(mm_plan_t P, const double* d_x, double* d_y, void* stream) {
  return guarded([&] {
    if (!P || !d_x || !d_y) fail(MM_EINVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    wait_ready(P, s);
    to_obs(P, d_x, P->vz, P->R, s);
    apply_H_obs(P, P->fs_main, P->vz, P->vq, P->y1, P->y2, P->R, s);
    to_glob(P, P->vq, d_y, P->R, s);
  });
}

mm_status_t mm_rhs(mm_plan_t P, const void* d_tod, int32_t tod_dtype, double* d_b, void* stream) {
  return guarded([&] {
    if (!P || !d_b || (!d_tod && P->n_t > 0)) fail(MM_EINVAL, "NULL argument");
    check_tod_dtype(tod_dtype);
    hipStream_t s = as_stream(stream);
    wait_ready(P, s);
    rhs_obs(P, P->fs_main, d_tod, tod_dtype == MM_F64, P->vq, P->y2, P->R, s);
    to_glob(P, P->vq, d_b, P->R, s);
  });
}

mm_status_t mm_solve(mm_plan_t P, const void* d_tod, int32_t tod_dtype, double* d_x,
                     const mm_solve_opts_t* opts, mm_solve_info_t* info, void* stream) {
  mm_status_t result = MM_OK;
  const mm_status_t st = guarded([&] {
    if (!P) fail(MM_EINVAL, "plan is NULL");
    check_tod_dtype(tod_dtype);
    RhsSource src;
    src.tod = d_tod;
    src.tod64 = tod_dtype == MM_F64;
    solve_impl(P, src, d_x, opts, info, as_stream(stream), &result);
    ++P->solves;
  });
  return st != MM_OK ? st : result;
}

mm_status_t mm_solve_rhs(mm_plan_t P, const double* d_b, double* d_x, const mm_solve_opts_t* opts,
                         mm_solve_info_t* info, void* stream) {
  mm_status_t result = MM_OK;
  const mm_status_t st = guarded([&] {
    if (!P || !d_b) fail(MM_EINVAL, "NULL argument");
    RhsSource src;
    src.map = d_b;
    solve_impl(P, src, d_x, opts, info, as_stream(stream), &result);
    ++P->solves;
  });
  return st != MM_OK ? st : result;
}

mm_status_t mm_noise_gradient(mm_plan_t P, const void* d_tod, int32_t tod_dtype, const double* d_m,
                              const double* d_lambda, double* grad_out, void* stream) {
  return guarded([&] {
    if (!P || !grad_out || !d_m || !d_lambda || (!d_tod && P->n_t > 0)) fail(MM_EINVAL, "NULL argument");
    check_tod_dtype(tod_dtype);
    if (!P->d_params) fail(MM_EUNSUPPORTED, "the plan was built from explicit lags: no noise parameters");
    hipStream_t s = as_stream(stream);
    wait_ready(P, s);
    const FilterSetup& f64 = P->main_fp64() ? P->fs_main : P->fs64;
    double* ya = P->main_fp64() ? (double*)P->y1 : P->y64a;   // d, then u = P lambda_r, in float64
    double* yb = P->main_fp64() ? (double*)P->y2 : P->y64b;   // dN^-1/dtheta v_r
    const bool in64 = tod_dtype == MM_F64;
    const int esz = in64 ? 8 : 4;
    const int nfl = P->n_filt, n_iv = std::max(P->n_iv, 1);
    const int64_t spec_n = (int64_t)nfl * (f64.N + 1);
    const int batch = std::max(1, std::min(nfl, 16));
    const size_t lsb = lags_scratch_bytes(P->n_c, P->lag_len, batch);
    // temporaries above the work vectors, released in reverse order on every exit
    double* v64 = P->temp<double>(std::max<int64_t>(P->n_t, 1));               // v_r = d_r - P m_r
    double* dlags = P->temp<double>((int64_t)nfl * P->n_c);
    double* dspec = P->temp<double>(3 * spec_n);                                   // one symbol per theta
    double* ivd = P->temp<double>(3 * (int64_t)n_iv);
    char* lscr = P->temp<char>((int64_t)std::max(lsb, symbol_scratch_bytes(f64.logn, true, nfl)));
    auto release_all = [&]() {
      P->release(lscr);
      P->release(ivd);
      P->release(dspec);
      P->release(dlags);
      P->release(v64);
    };
    std::vector<double> hd(3 * (size_t)n_iv);
    std::vector<double> grad((size_t)nfl * 3, 0.0);
    try {
      for (int mode = 1; mode <= 3; ++mode) {
        hipchk(launch_lags(P->d_params, nfl, P->f_samp, P->n_c, P->lag_len, dlags, lscr, lsb, s, mode),
               "derivative lags");
        build_symbols(f64, dlags, nfl, P->n_c, dspec + (mode - 1) * spec_n, lscr, s);
      }
      for (int r = 0; r < P->R; ++r) {
        // v_r = d_r - P m_r and u_r = P lambda_r, both in float64
        to_obs(P, d_m + (int64_t)r * P->ng(), P->vz, 1, s);
        gather_all(P, true, P->vz, v64, 1, s);
        hipchk(launch_convert(in64, true, (const char*)d_tod + (size_t)r * P->n_t * esz, ya, P->n_t, s), "convert");
        hipchk(launch_sub(v64, ya, v64, P->n_t, s), "residual TOD");
        to_obs(P, d_lambda + (int64_t)r * P->ng(), P->vz, 1, s);
        gather_all(P, true, P->vz, ya, 1, s);
        for (int mode = 0; mode < 3; ++mode) {
          apply_ols(P, f64, true, v64, yb, dspec + mode * spec_n, 1, s);
          hipchk(launch_interval_dots(ya, yb, P->d_iv_start, P->n_iv, ivd + (int64_t)mode * n_iv, s),
                 "interval dots");
        }
        hipchk(hipMemcpyAsync(hd.data(), ivd, sizeof(double) * 3 * n_iv, hipMemcpyDeviceToHost, s), "copy");
        hipchk(hipStreamSynchronize(s), "noise gradient");
        for (int mode = 0; mode < 3; ++mode)
          for (int b = 0; b < P->n_iv; ++b) grad[(size_t)P->iv_filter[b] * 3 + mode] += hd[(size_t)mode * n_iv + b];
      }
    } catch (...) {
      release_all();
      throw;
    }
    release_all();
    std::memcpy(grad_out, grad.data(), sizeof(double) * grad.size());
  });
}

mm_status_t mm_noise_lags_workspace_size(int32_t n_c, int64_t lag_dft_len, size_t* bytes) {
  return guarded([&] {
    if (!bytes) fail(MM_EINVAL, "bytes is NULL");
    static const double dummy = 0;
    *bytes = check_lag_args(&dummy, 1, 1.0, n_c, lag_dft_len, 0, &dummy);
  });
}

mm_status_t mm_noise_lags(const double* d_params, int32_t n_filters, double f_samp, int32_t n_c,
                          int64_t lag_dft_len, int32_t deriv, double* d_lags, void* d_ws, size_t ws_bytes,
                          void* stream) {
  return guarded([&] {
    const size_t need = check_lag_args(d_params, n_filters, f_samp, n_c, lag_dft_len, deriv, d_lags);
    if (!d_ws) fail(MM_EINVAL, "d_ws is NULL");
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) fail(MM_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
      fail(MM_EINVAL, "workspace of " + std::to_string(ws_bytes) + " bytes is below the " + std::to_string(need) +
                          " bytes mm_noise_lags_workspace_size gives");
    hipchk(launch_lags(d_params, n_filters, f_samp, n_c, lag_dft_len, d_lags, d_ws, ws_bytes, as_stream(stream), deriv),
           "lag construction");
  });
}

mm_status_t mm_noise_lags_noalloc(const double* d_params, int32_t n_filters, double f_samp, int32_t n_c,
                                  int64_t lag_dft_len, int32_t deriv, double* d_lags, void* stream) {
  return guarded([&] {
    const size_t need = check_lag_args(d_params, n_filters, f_samp, n_c, lag_dft_len, deriv, d_lags);
    if (need > kNoAllocScratchBytes)
      fail(MM_EINVAL, "this n_c and lag_dft_len need " + std::to_string(need) + " bytes of scratch, above the " +
                          std::to_string(kNoAllocScratchBytes) + " bytes of the allocation-free variant");
    hipchk(launch_lags(d_params, n_filters, f_samp, n_c, lag_dft_len, d_lags, noalloc_scratch(), kNoAllocScratchBytes,
                       as_stream(stream), deriv),
           "lag construction");
  });
}

int32_t mm_fft_length_rule(int32_t n_c, int64_t longest) { return fft_length_rule(n_c, longest); }

const char* mm_last_error(void) { return g_last_error.c_str(); }

const char* mm_version(void) { return "mm 0.1 (gfx950)"; }

}  // extern "C"
