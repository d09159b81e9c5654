// C ABI and host runtime of the matched-filter library (see include/bfsearch.h).
//
// A plan owns, for every segment length it accepts (the powers of two in
// [n_min, n]), the resident template bank at that length (the spectra of
// every template zero-padded to it, built on the device at plan time) and the
// FFT twiddle tables.  A job owns the per-call buffers (segment spectra,
// sigma, tail buffer and counter, segment table) which return to a per-plan
// pool on release, so steady-state filter calls do not allocate.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "bfsearch.h"
#include "bfs_kernelset.h"
#include "bfs_runtime_kernels.h"
#include "bfs_tail_sort.h"

using namespace bfs;

static_assert(sizeof(tail_rec) == sizeof(bfs_tail), "tail record layout");
static_assert(sizeof(tail_rec64) == sizeof(bfs_tail64), "tail record layout");
static_assert(sizeof(coinc_rec) == sizeof(bfs_coinc), "coincidence record layout");

namespace {

// Result-list heads a job publishes to pinned host memory at its end (tails:
// up to the count sorted on the host; projection entries; coincidences).
constexpr uint64_t PUB_TAILS = 1u << 15;
constexpr uint64_t PUB_PROJ = 1u << 17;
constexpr uint64_t PUB_COINC = 1u << 15;
constexpr int N_TILES = 5;
constexpr uint32_t TILES[N_TILES] = {1, 2, 4, 8, 16};

// Default segments per tile: as many segment spectra as fill half of one XCD's 4 MiB L2.
uint32_t default_tile(const KernelSet& ks) {
  const uint64_t row = uint64_t(ks.M) * 2 * ks.real_size;
  return uint32_t(std::max<uint64_t>(1, (2ull << 20) / row));
}

Candidates candidates(bfs_precision p, uint32_t m) {
  switch (p) {
    case BFS_FP64: return candidates_f64(m);
    case BFS_FP32: return candidates_f32(m);
    case BFS_FP32_W16F: return candidates_w16f(m);
    case BFS_FP32_W16B: return candidates_w16b(m);
  }
  return Candidates{};
}

const KernelSet* pick_kernels(bfs_precision p, uint32_t m) {
  const Candidates c = candidates(p, m);
  return c.count ? c.ks[0] : nullptr;
}

// ----------------------------------------------------------------- tables --
// exp(+2 pi i num / den) rounded from long double.
void twiddle(uint64_t num, uint64_t den, long double& c, long double& s) {
  const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)(num % den) / (long double)den;
  c = cosl(ang);
  s = sinl(ang);
}

uint64_t table_elems(const KernelSet& ks) {
  const uint64_t S1 = uint64_t(ks.R2) * ks.R3;
  return 2ull * (uint64_t(ks.M) + uint64_t(ks.FM) + S1);
}

template <typename T>
std::vector<T> make_tables(const KernelSet& ks, uint32_t n) {
  // layout: tw_u [M] (exp(2 pi i k / N)) | tw1 [R1][S1] | tw2 [R2][R3], interleaved (re, im)
  const uint32_t S1 = ks.R2 * ks.R3;
  std::vector<T> out(table_elems(ks));
  size_t o = 0;
  long double c, s;
  for (uint32_t k = 0; k < uint32_t(ks.M); ++k) {
    twiddle(k, n, c, s);
    out[o++] = T(c);
    out[o++] = T(s);
  }
  for (uint32_t n0 = 0; n0 < uint32_t(ks.R1); ++n0)
    for (uint32_t col = 0; col < S1; ++col) {
      twiddle(uint64_t(n0) * col, uint64_t(ks.FM), c, s);
      out[o++] = T(c);
      out[o++] = T(s);
    }
  for (uint32_t m0 = 0; m0 < uint32_t(ks.R2); ++m0)
    for (uint32_t j1 = 0; j1 < uint32_t(ks.R3); ++j1) {
      twiddle(uint64_t(m0) * j1, S1, c, s);
      out[o++] = T(c);
      out[o++] = T(s);
    }
  return out;
}

// numpy.linspace(lo, hi, n) element i: i*step + lo, the last element exactly hi
double linspace_at(double lo, double hi, uint32_t n, uint32_t i) {
#pragma clang fp contract(off)
  if (n == 1) return lo;
  if (i == n - 1) return hi;
  const double step = (hi - lo) / double(n - 1);
  const double prod = double(i) * step;
  return prod + lo;
}

bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

int log2u(uint64_t x) {
  int l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

// Capacities of a pooled set of job buffers.
struct JobNeed {
  uint64_t ybytes = 0;     // segment spectra, all groups
  uint64_t zbytes = 0;     // transform scratch of the split group (0 if none)
  uint64_t sigma = 0;      // S * K doubles
  uint64_t meta = 0;       // segment table bytes
  uint64_t proj = 0;       // projection entries (sum of segment lengths; 0: tail list)
  uint64_t coinc = 0;      // coincidence slots (sum of the pairs' lengths; 0: none)
};

struct JobBuffers {
  JobNeed cap;
  void* y = nullptr;
  void* z = nullptr;
  double* sigma = nullptr;
  void* tails = nullptr;  // device tail records of the plan's type (tail_rec or tail_rec64)
  unsigned long long* counter = nullptr;
  void* meta = nullptr;       // device segment table
  void* meta_host = nullptr;  // pinned host staging of the table
  unsigned long long* proj = nullptr;        // projection keys [sum of segment lengths]
  unsigned long long* plist = nullptr;       // compacted (index, key) pairs
  coinc_rec* clist = nullptr;                // coincidences of detector pairs
  unsigned long long* count_host = nullptr;  // pinned: the job's published counters (tails, projection, coincidences)
  void* tails_host = nullptr;                // pinned staging of fetched tails (the plan's records)
  uint64_t tails_host_cap = 0;
  // pinned, written by publish_kernel at the job's end: the first pub_* entries of each
  // list (never reallocated: captured graphs hold these addresses)
  void* pub_tails = nullptr;
  unsigned long long* pub_proj = nullptr;
  coinc_rec* pub_coinc = nullptr;
  uint64_t pub_tails_cap = 0, pub_proj_cap = 0, pub_coinc_cap = 0;
  void* dev_count_host = nullptr;  // device addresses of count_host and the pub_* buffers
  void* dev_pub_tails = nullptr;
  void* dev_pub_proj = nullptr;
  void* dev_pub_coinc = nullptr;
  void* sorted = nullptr;  // device: sorted tail records [sort_cap], then the sort's work area
  uint64_t sort_cap = 0;
  uint64_t sort_bytes = 0;
  // [0] job queued, [1]/[2] around the correlation kernels, [3] job done
  // after the publication of its results, [4] segment transforms done (orders
  // the correlation stream after them).  done = the event that completes the
  // job: 3, or 2 for dense correlations (nothing published).
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int done = 3;
  uint64_t bytes = 0;
  hipGraphExec_t gexec = nullptr;  // captured job body (graph plans)
  std::vector<uint64_t> gkey;      // the shape it was captured for
};

// One resident size of a plan.
struct SizePlan {
  uint32_t N = 0, M = 0;
  const KernelSet* ks = nullptr;  // the chosen candidate
  int cand = 0, n_cand = 0;
  float tuned_us[MAX_CANDIDATES] = {};  // measured us per correlation (autotuned plans)
  uint32_t tile = 1;                    // segments per tile of the workgroup order
  float tile_us[N_TILES] = {};          // measured us per correlation for TILES[i] (autotuned plans)
  void* bank = nullptr;
  void* tables = nullptr;
  const void* tw_u = nullptr;
  const void* tw1 = nullptr;
  const void* tw2 = nullptr;
  uint64_t bank_bytes = 0, tab_bytes = 0;
  uint32_t fused_rows = 0;  // fused plans: nonzero input rows of the forward transform's first pass
  // segment transforms split ks->join_a ways: the kernel set and tables of the length-1024
  // sub-transforms (null when the length's set has no join)
  const KernelSet* sub = nullptr;
  void* sub_tables = nullptr;
  const void* sub_tw1 = nullptr;
  const void* sub_tw2 = nullptr;
  uint64_t sub_tab_bytes = 0;
};

}  // namespace

struct bfs_plan {
  int device = 0;
  uint32_t n_max = 0, n_min = 0, K = 0;
  bfs_precision prec = BFS_FP32;
  double kappa = 0.0, kappa_hi = 0.0;
  uint64_t cap = 0;
  std::vector<SizePlan> sizes;  // ascending N: sizes[i].N = n_min << i
  size_t rec_bytes = sizeof(tail_rec);  // tail record the kernels write: 24 bytes for FP64, else 16
  uint32_t cus = 0;                     // compute units of the device
  uint64_t bank_bytes = 0, plan_bytes = 0, budget = 0;
  bool graph = false;
  bool project = false;  // per-lag max projection instead of the tail list
  bool pairs = false;    // segments come as detector pairs (2p, 2p + 1)
  // fused synthesis (no resident bank): the grid parameters of every template
  // (f0 [K] | fdot [K] doubles, len [K] u32) and their unit-norm factors [K]
  bool fused = false;
  void* fparams = nullptr;
  float* fnorm = nullptr;
  double fs = 0.0;
  int taper = 0, sym = 0;
  double delta = 0.0;    // coincidence window (Hz); 0: none
  double* f0_dev = nullptr;  // initial frequency of every template (coincidence plans)
  hipStream_t copy_stream = nullptr;
  hipStream_t capture_stream = nullptr;  // graph plans only
  std::mutex capture_mu;  // one capture at a time on capture_stream
  // Correlation stream paired with each caller stream that queued jobs: a
  // job's segment transforms run on the caller's stream, its correlation
  // kernels on the paired stream, so the next job's transforms overlap them.
  // At most MAX_CORR_STREAMS are created; later caller streams share them
  // (still correct: their fused kernels then run one after another).
  std::mutex stream_mu;
  std::vector<std::pair<hipStream_t, hipStream_t>> corr_streams;  // caller stream -> paired stream
  std::vector<hipStream_t> owned_streams;
  void* scratch = nullptr;  // this device's no-allocation scratch area (device address)
  std::mutex mu;
  std::vector<JobBuffers*> pool;  // released buffer sets (still allocated on the device)
  uint64_t pool_bytes = 0;         // their device bytes
  uint64_t live_job_bytes = 0;
  int live_jobs = 0;
};

namespace {

// Segments of one length within a job.
struct Group {
  const SizePlan* sp = nullptr;
  uint32_t count = 0;
  uint64_t y_off = 0;     // byte offset of the group's spectra in the job's y buffer
  uint64_t yf_off = 0;    // fused plans: byte offset of their copy in the fused layout
  uint32_t first = 0;     // index of the group's first entry in the segment table
};

}  // namespace

struct bfs_job {
  bfs_plan* plan = nullptr;
  JobBuffers* buf = nullptr;
  hipStream_t stream = nullptr;
  uint32_t S = 0;
  std::vector<Group> groups;
  std::vector<uint32_t> seg_len;  // per global segment
};

namespace {

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return BFS_ERR_HIP; \
  } while (0)

bfs_status alloc_checked(void** p, uint64_t bytes) {
  if (hipMalloc(p, bytes ? bytes : 256) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return BFS_ERR_OUT_OF_MEMORY;
  }
  return BFS_OK;
}

void free_job_buffers(JobBuffers* b) {
  if (!b) return;
  for (void* q : {b->y, b->z, static_cast<void*>(b->sigma), static_cast<void*>(b->tails),
                  static_cast<void*>(b->counter), b->meta, static_cast<void*>(b->proj), static_cast<void*>(b->plist),
                  static_cast<void*>(b->clist)})
    if (q) (void)hipFree(q);
  if (b->meta_host) (void)hipHostFree(b->meta_host);
  if (b->count_host) (void)hipHostFree(b->count_host);
  if (b->pub_tails) (void)hipHostFree(b->pub_tails);
  if (b->pub_proj) (void)hipHostFree(b->pub_proj);
  if (b->pub_coinc) (void)hipHostFree(b->pub_coinc);
  if (b->tails_host) (void)hipHostFree(b->tails_host);
  if (b->sorted) (void)hipFree(b->sorted);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  for (auto& e : b->ev)
    if (e) (void)hipEventDestroy(e);
  delete b;
}

void free_plan(bfs_plan* p) {
  if (!p) return;
  for (auto* b : p->pool) free_job_buffers(b);
  p->pool.clear();
  for (auto& sp : p->sizes) {
    if (sp.bank) (void)hipFree(sp.bank);
    if (sp.tables) (void)hipFree(sp.tables);
    if (sp.sub_tables) (void)hipFree(sp.sub_tables);
  }
  if (p->f0_dev) (void)hipFree(p->f0_dev);
  if (p->fparams) (void)hipFree(p->fparams);
  if (p->fnorm) (void)hipFree(p->fnorm);
  if (p->copy_stream) (void)hipStreamDestroy(p->copy_stream);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  for (hipStream_t cs : p->owned_streams) (void)hipStreamDestroy(cs);
  delete p;
}

uint32_t n_min_of(const bfs_plan_desc* d) { return d->n_min ? d->n_min : d->n; }

// The candidate of length n / 2 with a fused-synthesis kernel (or -1).
int fused_candidate(bfs_precision p, uint32_t m) {
  const Candidates c = candidates(p, m);
  for (int i = 0; i < c.count; ++i)
    if (c.ks[i]->corr_fused) return i;
  return -1;
}

// Fused synthesis serves grid plans of FP32 precision, single segments, at
// lengths whose transform has a fused kernel.
bool fused_possible(const bfs_plan_desc* d) {
  if (d->explicit_templates || d->precision != BFS_FP32 || (d->flags & BFS_PLAN_PAIRS)) return false;
  for (uint32_t n = n_min_of(d); n <= d->n; n <<= 1)
    if (fused_candidate(d->precision, n / 2) < 0) return false;
  return true;
}

bfs_status validate(const bfs_plan_desc* d) {
  if (!d) return BFS_ERR_INVALID_ARG;
  if (!is_pow2(d->n) || d->n < 2) return BFS_ERR_INVALID_ARG;
  const uint32_t nmin = n_min_of(d);
  if (!is_pow2(nmin) || nmin < 2 || nmin > d->n) return BFS_ERR_INVALID_ARG;
  if (!(d->fs > 0.0) || !std::isfinite(d->fs)) return BFS_ERR_INVALID_ARG;
  if (!(d->kappa >= 0.0) || !std::isfinite(d->kappa)) return BFS_ERR_INVALID_ARG;
  if (d->tail_capacity < 1) return BFS_ERR_INVALID_ARG;
  if (d->precision < BFS_FP64 || d->precision > BFS_FP32_W16B) return BFS_ERR_INVALID_ARG;
  if (d->taper > 1) return BFS_ERR_INVALID_ARG;
  if (d->flags & ~uint32_t(BFS_PLAN_GRAPH | BFS_PLAN_AUTOTUNE | BFS_PLAN_PROJECT | BFS_PLAN_SYMMETRIC | BFS_PLAN_PAIRS |
                           BFS_PLAN_FUSED))
    return BFS_ERR_INVALID_ARG;
  if (!std::isfinite(d->coinc_delta_hz) || d->coinc_delta_hz < 0.0) return BFS_ERR_INVALID_ARG;
  if (d->coinc_delta_hz > 0.0 && (!(d->flags & BFS_PLAN_PAIRS) || !(d->flags & BFS_PLAN_PROJECT) ||
                                  d->explicit_templates))
    return BFS_ERR_INVALID_ARG;
  if (!std::isfinite(d->kappa_hi) || (d->kappa_hi != 0.0 && !(d->kappa_hi > d->kappa))) return BFS_ERR_INVALID_ARG;
  if (d->candidate > uint32_t(MAX_CANDIDATES)) return BFS_ERR_INVALID_ARG;
  if (d->tile > 65535) return BFS_ERR_INVALID_ARG;
  if (d->explicit_templates) {
    if (d->n_explicit < 1 || d->explicit_len < 1 || d->explicit_len > nmin) return BFS_ERR_INVALID_ARG;
  } else {
    if (d->n_f0 < 1 || d->n_fdot < 1) return BFS_ERR_INVALID_ARG;
    if (uint64_t(d->n_f0) * d->n_fdot > 0xffffffffull) return BFS_ERR_INVALID_ARG;
    if (d->n_tau < 1 || !d->tau) return BFS_ERR_INVALID_ARG;
    for (double v : {d->f0_lo, d->f0_hi, d->fdot_lo, d->fdot_hi})
      if (!std::isfinite(v)) return BFS_ERR_INVALID_ARG;
    for (uint32_t i = 0; i < d->n_tau; ++i) {
      if (!(d->tau[i] > 0.0) || !std::isfinite(d->tau[i])) return BFS_ERR_INVALID_ARG;
      const double L = std::nearbyint(d->tau[i] * d->fs);
      if (L < 1.0 || L > double(nmin)) return BFS_ERR_INVALID_ARG;
    }
  }
  for (uint32_t n = nmin; n <= d->n; n <<= 1) {
    const KernelSet* ks = pick_kernels(d->precision, n / 2);
    if (!ks) return BFS_ERR_UNSUPPORTED;
    if ((d->flags & BFS_PLAN_PAIRS) && !ks->corr_pair) return BFS_ERR_UNSUPPORTED;
  }
  if ((d->flags & BFS_PLAN_FUSED) && !fused_possible(d)) return BFS_ERR_UNSUPPORTED;
  return BFS_OK;
}

// Twiddle tables of kernel set ks into the size's table buffer (sized for
// every candidate), and the pointers into it.
bfs_status set_tables(SizePlan& sp, const KernelSet* ks) {
  const uint64_t bytes = table_elems(*ks) * ks->real_size;
  hipError_t e;
  if (ks->real_size == sizeof(double)) {
    auto tab = make_tables<double>(*ks, sp.N);
    e = hipMemcpy(sp.tables, tab.data(), bytes, hipMemcpyHostToDevice);
  } else {
    auto tab = make_tables<float>(*ks, sp.N);
    e = hipMemcpy(sp.tables, tab.data(), bytes, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return BFS_ERR_HIP;
  const char* tb = static_cast<const char*>(sp.tables);
  sp.ks = ks;
  sp.tw_u = tb;
  sp.tw1 = tb + 2ull * sp.M * ks->real_size;
  sp.tw2 = tb + 2ull * (uint64_t(sp.M) + uint64_t(ks->FM)) * ks->real_size;
  return BFS_OK;
}

// Tables of the length-1024 sub-transforms of a split segment transform
// (their own length 2048 as a real transform).
bfs_status set_sub_tables(SizePlan& sp) {
  const KernelSet& ks = *sp.sub;
  bfs_status st = alloc_checked(&sp.sub_tables, sp.sub_tab_bytes);
  if (st != BFS_OK) return st;
  hipError_t e;
  if (ks.real_size == sizeof(double)) {
    auto tab = make_tables<double>(ks, 2048);
    e = hipMemcpy(sp.sub_tables, tab.data(), sp.sub_tab_bytes, hipMemcpyHostToDevice);
  } else {
    auto tab = make_tables<float>(ks, 2048);
    e = hipMemcpy(sp.sub_tables, tab.data(), sp.sub_tab_bytes, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return BFS_ERR_HIP;
  const char* tb = static_cast<const char*>(sp.sub_tables);
  sp.sub_tw1 = tb + 2ull * ks.M * ks.real_size;
  sp.sub_tw2 = tb + 2ull * (uint64_t(ks.M) + uint64_t(ks.FM)) * ks.real_size;
  return BFS_OK;
}

// Queue the forward transform of `count` segments of one length into the
// packed half spectra y ([count][M]): segment i's samples at seg_ptr[i], or
// src + i src_stride when seg_ptr is null.  Lengths whose set joins split
// transforms run as count x join_a length-1024 transforms (many small
// workgroups instead of one large one per segment), the join and the unpack;
// the others as one workgroup per segment (two halves at the split length)
// and the unpack.  z: scratch of the same size as y (split and joined paths).
bfs_status queue_segment_fft(const SizePlan& sp, uint32_t count, const uint64_t* seg_ptr, const void* src,
                             uint64_t src_stride, void* y, void* z, hipStream_t st,
                             unsigned long long* zero = nullptr) {
  const KernelSet& ks = *sp.ks;
  FwdArgs a{};
  a.zero = zero;
  a.seg_ptr = seg_ptr;
  a.src = src;
  a.src_stride = src_stride;
  if (ks.join && sp.sub) {
    a.tw1 = sp.sub_tw1;
    a.tw2 = sp.sub_tw2;
    a.out = z;
    a.zs = uint32_t(ks.join_a);
    HIP_TRY(sp.sub->fwd(SRC_SAMPLES, count * uint32_t(ks.join_a), st, a));
    HIP_TRY(ks.join(count, st, z, y, sp.tw_u));
    HIP_TRY(ks.unpack_y(count, st, y, y, sp.tw_u));
    return BFS_OK;
  }
  a.tw1 = sp.tw1;
  a.tw2 = sp.tw2;
  a.out = ks.split ? z : y;
  HIP_TRY(ks.fwd(SRC_SAMPLES, count, st, a));
  HIP_TRY(ks.unpack_y(count, st, a.out, y, sp.tw_u));
  return BFS_OK;
}

// Autotuner: time every candidate kernel set of one size on the resident bank
// (up to 4096 templates against a zero segment spectrum: the work of a
// correlation does not depend on the data, only the rare tail writes do),
// best of three launches each, and keep the fastest; then, with that kernel,
// time every segment tile of the workgroup order on 16 segments.
bfs_status tune_size(bfs_plan* p, SizePlan& sp) {
  const Candidates c = candidates(p->prec, sp.M);
  const uint32_t Kt = std::min<uint32_t>(p->K, 4096);
  void* y = nullptr;
  void* tails = nullptr;
  void* counter = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const uint64_t ybytes = uint64_t(sp.M) * 2 * sp.ks->real_size;
  bfs_status st = alloc_checked(&y, ybytes);
  if (st == BFS_OK) st = alloc_checked(&tails, sizeof(tail_rec64));
  if (st == BFS_OK) st = alloc_checked(&counter, 256);
  if (st == BFS_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = BFS_ERR_HIP;
  hipStream_t s = p->copy_stream;
  if (st == BFS_OK && hipMemsetAsync(y, 0, ybytes, s) != hipSuccess) st = BFS_ERR_HIP;
  int best = 0;
  float best_ms = 0.f;
  for (int i = 0; i < c.count && c.count > 1 && st == BFS_OK; ++i) {
    st = set_tables(sp, c.ks[i]);
    if (st != BFS_OK) break;
    CorrArgs a{};
    a.bank = sp.bank;
    a.y = y;
    a.tw_u = sp.tw_u;
    a.tw1 = sp.tw1;
    a.tw2 = sp.tw2;
    a.K = Kt;
    a.kappa = p->kappa;
    a.tails = tails;
    a.counter = static_cast<unsigned long long*>(counter);
    a.cap = 1;
    a.cus = p->cus;
    float ms_min = 0.f;
    for (int r = 0; r < 4 && st == BFS_OK; ++r) {
      if (hipEventRecord(e0, s) != hipSuccess || c.ks[i]->corr(false, 1, s, a) != hipSuccess ||
          hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        st = BFS_ERR_HIP;
        break;
      }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = BFS_ERR_HIP;
      if (r == 1 || (r > 1 && ms < ms_min)) ms_min = ms;  // launch 0 warms up
    }
    sp.tuned_us[i] = ms_min * 1000.f / float(Kt);
    if (i == 0 || ms_min < best_ms) {
      best = i;
      best_ms = ms_min;
    }
  }
  if (st == BFS_OK) {
    st = set_tables(sp, c.ks[best]);
    sp.cand = best;
  }
  if (y) (void)hipFree(y);
  y = nullptr;
  // tile of the workgroup order, timed on TUNE_SEGS zero segment spectra
  constexpr uint32_t TUNE_SEGS = 16;
  if (st == BFS_OK) st = alloc_checked(&y, TUNE_SEGS * ybytes);
  if (st == BFS_OK && hipMemsetAsync(y, 0, TUNE_SEGS * ybytes, s) != hipSuccess) st = BFS_ERR_HIP;
  float best_tile_ms = 0.f;
  for (int i = 0; i < N_TILES && st == BFS_OK; ++i) {
    CorrArgs a{};
    a.bank = sp.bank;
    a.y = y;
    a.tw_u = sp.tw_u;
    a.tw1 = sp.tw1;
    a.tw2 = sp.tw2;
    a.K = Kt;
    a.tile = TILES[i];
    a.kappa = p->kappa;
    a.tails = tails;
    a.counter = static_cast<unsigned long long*>(counter);
    a.cap = 1;
    a.cus = p->cus;
    float ms_min = 0.f;
    for (int r = 0; r < 4 && st == BFS_OK; ++r) {
      if (hipEventRecord(e0, s) != hipSuccess || sp.ks->corr(false, TUNE_SEGS, s, a) != hipSuccess ||
          hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        st = BFS_ERR_HIP;
        break;
      }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = BFS_ERR_HIP;
      if (r == 1 || (r > 1 && ms < ms_min)) ms_min = ms;
    }
    sp.tile_us[i] = ms_min * 1000.f / float(Kt * TUNE_SEGS);
    if (i == 0 || ms_min < best_tile_ms) best_tile_ms = ms_min;
  }
  // The largest tile within 2 % of the fastest: timed on a slice of the bank,
  // tiles that differ by noise there differ at full size, where each pass of a
  // smaller tile reads the whole bank from HBM again (a 2^17 bank of 65,536
  // chirps is 32 GiB).
  for (int i = 0; i < N_TILES && st == BFS_OK; ++i)
    if (sp.tile_us[i] * float(Kt * TUNE_SEGS) <= 1.02f * best_tile_ms * 1000.f) sp.tile = TILES[i];
  if (y) (void)hipFree(y);
  if (tails) (void)hipFree(tails);
  if (counter) (void)hipFree(counter);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return st;
}

// Template spectra at every size: per chunk of templates, synthesis (or the
// explicit samples) + forward transform into scratch, then unpack + scale
// into the bank rows.
bfs_status build_banks(bfs_plan* p, const bfs_plan_desc* d) {
  const uint32_t K = p->K;
  const bool expl = d->explicit_templates != nullptr;
  std::vector<double> f0, fdot;
  std::vector<uint32_t> len;
  void* params = nullptr;
  uint64_t param_bytes = 0;
  if (expl) {
    param_bytes = uint64_t(d->n_explicit) * d->explicit_len * sizeof(double);
  } else {
    f0.resize(K);
    fdot.resize(K);
    len.resize(K);
    for (uint32_t j = 0; j < K; ++j) {
      f0[j] = linspace_at(d->f0_lo, d->f0_hi, d->n_f0, j / d->n_fdot);
      fdot[j] = linspace_at(d->fdot_lo, d->fdot_hi, d->n_fdot, j % d->n_fdot);
      len[j] = uint32_t(std::nearbyint(d->tau[j % d->n_tau] * d->fs));
    }
    param_bytes = uint64_t(K) * (2 * sizeof(double) + sizeof(uint32_t));
  }
  // scratch for the complex transforms of a chunk of templates at the largest
  // size, plus two energy sums per template
  const uint64_t row_bytes = uint64_t(p->n_max / 2) * 2 * p->sizes.back().ks->real_size;
  const uint64_t avail = p->budget > p->plan_bytes + param_bytes ? p->budget - p->plan_bytes - param_bytes : 0;
  if (avail < row_bytes + 16) return BFS_ERR_OUT_OF_MEMORY;
  const uint64_t chunk = std::min<uint64_t>(K, std::max<uint64_t>(1, std::min<uint64_t>(4096, avail / (2 * row_bytes + 16))));
  void* scratch = nullptr;
  double* energy = nullptr;
  bfs_status st = alloc_checked(&params, param_bytes);
  if (st != BFS_OK) return st;
  st = alloc_checked(&scratch, chunk * row_bytes);
  if (st == BFS_OK) st = alloc_checked(reinterpret_cast<void**>(&energy), 2 * chunk * sizeof(double));
  hipStream_t s = p->copy_stream;
  bfs_status out = st;
  if (st == BFS_OK) {
    out = BFS_ERR_HIP;
    do {
      const double* df0 = nullptr;
      const double* dfd = nullptr;
      const uint32_t* dlen = nullptr;
      if (expl) {
        if (hipMemcpyAsync(params, d->explicit_templates, param_bytes, hipMemcpyHostToDevice, s) != hipSuccess) break;
      } else {
        char* base = static_cast<char*>(params);
        if (hipMemcpyAsync(base, f0.data(), K * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess) break;
        if (hipMemcpyAsync(base + K * sizeof(double), fdot.data(), K * sizeof(double), hipMemcpyHostToDevice, s) !=
            hipSuccess)
          break;
        if (hipMemcpyAsync(base + 2 * K * sizeof(double), len.data(), K * sizeof(uint32_t), hipMemcpyHostToDevice, s) !=
            hipSuccess)
          break;
        df0 = reinterpret_cast<const double*>(base);
        dfd = reinterpret_cast<const double*>(base + K * sizeof(double));
        dlen = reinterpret_cast<const uint32_t*>(base + 2 * K * sizeof(double));
      }
      bool ok = true;
      for (const SizePlan& sp : p->sizes) {
        for (uint64_t j0 = 0; j0 < K && ok; j0 += chunk) {
          const uint32_t nb = uint32_t(std::min<uint64_t>(chunk, K - j0));
          FwdArgs a{};
          a.src = params;
          a.src_stride = expl ? d->explicit_len : 0;
          a.src_len = expl ? d->explicit_len : 0;
          a.f0 = df0;
          a.fdot = dfd;
          a.len = dlen;
          a.fs = d->fs;
          a.taper = int(d->taper);
          a.first = uint32_t(j0);
          a.tw1 = sp.tw1;
          a.tw2 = sp.tw2;
          a.out = scratch;
          a.energy = energy;
          const int src = expl ? SRC_EXPLICIT : ((d->flags & BFS_PLAN_SYMMETRIC) ? SRC_CHIRP_SYM : SRC_CHIRP);
          ok = sp.ks->fwd(src, nb, s, a) == hipSuccess;
          ok = ok && sp.ks->unpack_bank(nb, s, scratch, sp.bank, expl ? nullptr : energy, sp.tw_u, j0) == hipSuccess;
        }
      }
      if (!ok) break;
      if (hipStreamSynchronize(s) != hipSuccess) break;
      out = BFS_OK;
    } while (false);
  }
  if (params) (void)hipFree(params);
  if (scratch) (void)hipFree(scratch);
  if (energy) (void)hipFree(energy);
  return out;
}

// Per accepted length: the kernel set, tile and bytes of the plan; with fused
// synthesis no bank is kept (the candidate with a fused kernel, the grid
// parameters and unit-norm factors instead).
void size_plans(bfs_plan* p, const bfs_plan_desc* d, bool fused) {
  p->sizes.clear();
  p->fused = fused;
  p->bank_bytes = 0;
  p->plan_bytes = 0;
  uint32_t lmax = 0;
  if (!d->explicit_templates)
    for (uint32_t i = 0; i < d->n_tau; ++i) lmax = std::max(lmax, uint32_t(std::nearbyint(d->tau[i] * d->fs)));
  for (uint32_t n = p->n_min; n <= p->n_max; n <<= 1) {
    SizePlan sp;
    sp.N = n;
    sp.M = n / 2;
    const Candidates c = candidates(d->precision, sp.M);
    sp.cand = (d->candidate && int(d->candidate) <= c.count) ? int(d->candidate) - 1 : 0;
    if (fused) sp.cand = fused_candidate(d->precision, sp.M);
    sp.ks = c.ks[sp.cand];
    sp.n_cand = c.count;
    sp.tile = d->tile ? d->tile : default_tile(*sp.ks);
    sp.bank_bytes = fused ? 0 : uint64_t(p->K) * sp.M * sp.ks->spec_size;
    if (fused) {
      const uint32_t s1 = uint32_t(sp.ks->R2 * sp.ks->R3);
      sp.fused_rows = std::max<uint32_t>(1, ((lmax + 1) / 2 + s1 - 1) / s1);
    }
    for (int i = 0; i < c.count; ++i)
      sp.tab_bytes = std::max<uint64_t>(sp.tab_bytes, table_elems(*c.ks[i]) * c.ks[i]->real_size);
    if (sp.ks->join) {
      sp.sub = pick_kernels(d->precision, 1024);
      if (sp.sub) sp.sub_tab_bytes = table_elems(*sp.sub) * sp.sub->real_size;
    }
    p->bank_bytes += sp.bank_bytes;
    p->plan_bytes += sp.bank_bytes + sp.tab_bytes + sp.sub_tab_bytes;
    p->sizes.push_back(sp);
  }
  if (fused) p->plan_bytes += uint64_t(p->K) * (2 * sizeof(double) + sizeof(uint32_t) + sizeof(float));
}

// Fused plans: the grid parameters of every template on the device, and each
// template's unit-norm factor 1 / sqrt(sum w^2) from its FP64 samples.
bfs_status build_fused(bfs_plan* p, const bfs_plan_desc* d) {
  const uint32_t K = p->K;
  std::vector<double> f0(K), fdot(K);
  std::vector<uint32_t> len(K);
  for (uint32_t j = 0; j < K; ++j) {
    f0[j] = linspace_at(d->f0_lo, d->f0_hi, d->n_f0, j / d->n_fdot);
    fdot[j] = linspace_at(d->fdot_lo, d->fdot_hi, d->n_fdot, j % d->n_fdot);
    len[j] = uint32_t(std::nearbyint(d->tau[j % d->n_tau] * d->fs));
  }
  p->fs = d->fs;
  p->taper = int(d->taper);
  p->sym = (d->flags & BFS_PLAN_SYMMETRIC) ? 1 : 0;
  bfs_status st = alloc_checked(&p->fparams, uint64_t(K) * (2 * sizeof(double) + sizeof(uint32_t)));
  if (st == BFS_OK) st = alloc_checked(reinterpret_cast<void**>(&p->fnorm), uint64_t(K) * sizeof(float));
  if (st != BFS_OK) return st;
  char* base = static_cast<char*>(p->fparams);
  hipStream_t s = p->copy_stream;
  HIP_TRY(hipMemcpyAsync(base, f0.data(), K * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + K * sizeof(double), fdot.data(), K * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + 2ull * K * sizeof(double), len.data(), K * sizeof(uint32_t), hipMemcpyHostToDevice, s));
  const auto* df0 = reinterpret_cast<const double*>(base);
  const auto* dfd = df0 + K;
  const auto* dlen = reinterpret_cast<const uint32_t*>(df0 + 2ull * K);
  constexpr uint32_t CHUNK = 1u << 24;  // templates per launch (one workgroup each)
  for (uint32_t j0 = 0; j0 < K; j0 += CHUNK) {
    const uint32_t nb = std::min(CHUNK, K - j0);
    hipLaunchKernelGGL(chirp_norm_kernel, dim3(nb), dim3(256), 0, s, df0 + j0, dfd + j0, dlen + j0, p->fs, p->taper,
                       p->sym, p->fnorm + j0);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(s));
  return BFS_OK;
}

bool covers(const JobNeed& c, const JobNeed& n) {
  return c.ybytes >= n.ybytes && c.zbytes >= n.zbytes && c.sigma >= n.sigma && c.meta >= n.meta && c.proj >= n.proj &&
         c.coinc >= n.coinc;
}

uint64_t need_bytes(const JobNeed& c, uint64_t cap, size_t rec_bytes) {
  return c.ybytes + c.zbytes + c.sigma * sizeof(double) + cap * rec_bytes + c.meta + 3 * 8 * c.proj +
         c.coinc * sizeof(coinc_rec) + 256;
}

bfs_status get_job_buffers(bfs_plan* p, const JobNeed& need, JobBuffers** out) {
  std::lock_guard<std::mutex> lk(p->mu);
  for (size_t i = 0; i < p->pool.size(); ++i) {
    if (covers(p->pool[i]->cap, need)) {
      *out = p->pool[i];
      p->pool.erase(p->pool.begin() + long(i));
      p->pool_bytes -= (*out)->bytes;
      p->live_job_bytes += (*out)->bytes;
      ++p->live_jobs;
      return BFS_OK;
    }
  }
  JobNeed c = need;
  for (auto* b : p->pool) {  // grow to cover what the pooled sets covered
    c.ybytes = std::max(c.ybytes, b->cap.ybytes);
    c.zbytes = std::max(c.zbytes, b->cap.zbytes);
    c.sigma = std::max(c.sigma, b->cap.sigma);
    c.meta = std::max(c.meta, b->cap.meta);
    c.proj = std::max(c.proj, b->cap.proj);
    c.coinc = std::max(c.coinc, b->cap.coinc);
  }
  uint64_t bytes = need_bytes(c, p->cap, p->rec_bytes);
  if (p->plan_bytes + p->live_job_bytes + bytes > p->budget) {
    c = need;  // the minimal set, after dropping the pool
    bytes = need_bytes(c, p->cap, p->rec_bytes);
  }
  for (auto* b : p->pool) free_job_buffers(b);
  p->pool.clear();
  p->pool_bytes = 0;
  if (p->plan_bytes + p->live_job_bytes + bytes > p->budget) return BFS_ERR_OUT_OF_MEMORY;
  auto* b = new (std::nothrow) JobBuffers();
  if (!b) return BFS_ERR_OUT_OF_MEMORY;
  b->cap = c;
  b->bytes = bytes;
  bfs_status st = alloc_checked(&b->y, c.ybytes);
  if (st == BFS_OK && c.zbytes) st = alloc_checked(&b->z, c.zbytes);
  if (st == BFS_OK) st = alloc_checked(reinterpret_cast<void**>(&b->sigma), c.sigma * sizeof(double));
  if (st == BFS_OK) st = alloc_checked(&b->tails, p->cap * p->rec_bytes);
  if (st == BFS_OK) st = alloc_checked(reinterpret_cast<void**>(&b->counter), 256);
  if (st == BFS_OK) st = alloc_checked(&b->meta, c.meta);
  if (st == BFS_OK && c.proj) st = alloc_checked(reinterpret_cast<void**>(&b->proj), c.proj * 8);
  if (st == BFS_OK && c.proj) st = alloc_checked(reinterpret_cast<void**>(&b->plist), c.proj * 16);
  if (st == BFS_OK && c.coinc) st = alloc_checked(reinterpret_cast<void**>(&b->clist), c.coinc * sizeof(coinc_rec));
  if (st == BFS_OK && (hipHostMalloc(&b->meta_host, c.meta ? c.meta : 256, hipHostMallocDefault) != hipSuccess ||
                       hipHostMalloc(reinterpret_cast<void**>(&b->count_host), 256, hipHostMallocDefault) !=
                           hipSuccess)) {
    (void)hipGetLastError();
    st = BFS_ERR_OUT_OF_MEMORY;
  }
  if (st == BFS_OK) {
    b->pub_tails_cap = std::min<uint64_t>(p->cap, PUB_TAILS);
    b->pub_proj_cap = std::min<uint64_t>(c.proj, PUB_PROJ);
    b->pub_coinc_cap = std::min<uint64_t>(c.coinc, PUB_COINC);
    if ((b->pub_tails_cap && hipHostMalloc(&b->pub_tails, b->pub_tails_cap * p->rec_bytes, hipHostMallocDefault) !=
                                 hipSuccess) ||
        (b->pub_proj_cap && hipHostMalloc(reinterpret_cast<void**>(&b->pub_proj), b->pub_proj_cap * 16,
                                          hipHostMallocDefault) != hipSuccess) ||
        (b->pub_coinc_cap && hipHostMalloc(reinterpret_cast<void**>(&b->pub_coinc),
                                           b->pub_coinc_cap * sizeof(coinc_rec), hipHostMallocDefault) != hipSuccess)) {
      (void)hipGetLastError();
      st = BFS_ERR_OUT_OF_MEMORY;
    }
  }
  if (st == BFS_OK) {
    auto dev = [](void* h, void** d) { return !h || hipHostGetDevicePointer(d, h, 0) == hipSuccess; };
    if (!dev(b->count_host, &b->dev_count_host) || !dev(b->pub_tails, &b->dev_pub_tails) ||
        !dev(b->pub_proj, &b->dev_pub_proj) || !dev(b->pub_coinc, &b->dev_pub_coinc)) {
      (void)hipGetLastError();
      st = BFS_ERR_HIP;
    }
  }
  for (int i = 0; i < 4 && st == BFS_OK; ++i)
    if (hipEventCreate(&b->ev[i]) != hipSuccess) st = BFS_ERR_HIP;
  if (st == BFS_OK && hipEventCreateWithFlags(&b->ev[4], hipEventDisableTiming) != hipSuccess) st = BFS_ERR_HIP;
  if (st != BFS_OK) {
    free_job_buffers(b);
    return st;
  }
  p->live_job_bytes += b->bytes;
  ++p->live_jobs;
  *out = b;
  return BFS_OK;
}

void put_job_buffers(bfs_plan* p, JobBuffers* b) {
  std::lock_guard<std::mutex> lk(p->mu);
  p->live_job_bytes -= b->bytes;
  --p->live_jobs;
  p->pool.push_back(b);
  p->pool_bytes += b->bytes;
}

const SizePlan* size_plan(const bfs_plan* p, uint32_t n) {
  if (!is_pow2(n) || n < p->n_min || n > p->n_max) return nullptr;
  return &p->sizes[size_t(log2u(n) - log2u(p->n_min))];
}

// A prepared job: segments grouped by length (longest first), the segment
// table (device addresses and global ids per group) staged in pinned memory.
struct Layout {
  std::vector<Group> groups;
  std::vector<uint32_t> seg_len;
  JobNeed need;
};

// Bytes of the segment table of S segments (see stage_table).
uint64_t table_bytes(uint32_t S) { return uint64_t(S) * (3 * sizeof(uint64_t) + sizeof(uint32_t)) + sizeof(uint64_t); }

bfs_status make_layout(const bfs_plan* p, const uint32_t* lens, uint32_t S, Layout& L) {
  L.seg_len.resize(S);
  for (uint32_t s = 0; s < S; ++s) {
    const uint32_t n = lens ? lens[s] : p->n_max;
    if (!size_plan(p, n)) return BFS_ERR_INVALID_ARG;
    L.seg_len[s] = n;
  }
  if (p->pairs) {  // channels 2q and 2q + 1 of every pair, of equal length
    if (S & 1u) return BFS_ERR_INVALID_ARG;
    for (uint32_t s = 0; s < S; s += 2)
      if (L.seg_len[s] != L.seg_len[s + 1]) return BFS_ERR_INVALID_ARG;
  }
  uint64_t ybytes = 0, zbytes = 0, first = 0;
  for (int i = int(p->sizes.size()) - 1; i >= 0; --i) {
    const SizePlan& sp = p->sizes[size_t(i)];
    uint32_t cnt = 0;
    for (uint32_t s = 0; s < S; ++s) cnt += (L.seg_len[s] == sp.N);
    if (!cnt) continue;
    Group g;
    g.sp = &sp;
    g.count = cnt;
    g.y_off = ybytes;
    g.first = uint32_t(first);
    const uint64_t gbytes = uint64_t(cnt) * sp.M * 2 * sp.ks->real_size;
    ybytes += (gbytes + 255) & ~uint64_t(255);
    if (sp.ks->split || (sp.ks->join && sp.sub)) zbytes = std::max(zbytes, gbytes);
    first += cnt;
    L.groups.push_back(g);
  }
  if (p->fused) {  // a second copy of every group's spectra, in the fused layout
    for (Group& g : L.groups) g.yf_off = ybytes + g.y_off;
    ybytes *= 2;
  }
  L.need.ybytes = ybytes;
  L.need.zbytes = zbytes;
  L.need.sigma = uint64_t(S) * p->K;
  L.need.meta = table_bytes(S) + 256;
  if (p->project)
    for (uint32_t s = 0; s < S; ++s) L.need.proj += L.seg_len[s];
  if (p->delta > 0.0)
    for (uint32_t s = 0; s < S; s += 2) L.need.coinc += L.seg_len[s];
  return BFS_OK;
}

// Fill the pinned segment table: per entry in group order [S] device address
// of the samples and [S] offset of the segment's lags in the projection keys
// (segments back to back in the caller's order); [S + 1] those offsets in the
// caller's order (the last is the total); per entry in group order [S] caller
// index.
void stage_table(const bfs_plan* p, const void* y_dev, const uint64_t* offs, const Layout& L, void* host) {
  const uint32_t S = uint32_t(L.seg_len.size());
  auto* ptrs = static_cast<uint64_t*>(host);
  auto* poff = ptrs + S;
  auto* lag0c = poff + S;
  auto* ids = reinterpret_cast<uint32_t*>(lag0c + S + 1);
  const size_t rs = p->sizes[0].ks->real_size;
  std::vector<uint64_t> off(S), lag0(S);
  uint64_t acc = 0;
  for (uint32_t s = 0; s < S; ++s) {
    off[s] = offs ? offs[s] : acc;
    lag0[s] = acc;
    lag0c[s] = acc;
    acc += L.seg_len[s];
  }
  lag0c[S] = acc;
  for (const Group& g : L.groups) {
    uint32_t k = g.first;
    for (uint32_t s = 0; s < S; ++s) {
      if (L.seg_len[s] != g.sp->N) continue;
      ptrs[k] = uint64_t(reinterpret_cast<uintptr_t>(y_dev)) + off[s] * rs;
      poff[k] = lag0[s];
      ids[k] = s;
      ++k;
    }
  }
}

// Queue the first part of a job on st: the projection-key reset, the table
// upload, the segment transforms of every group (the first also clears the
// job's counters).
bfs_status enqueue_prep(bfs_plan* p, JobBuffers* b, const Layout& L, bool dense, hipStream_t st) {
  const uint32_t S = uint32_t(L.seg_len.size());
  const bool project = p->project && !dense;
  if (project) {
    const uint64_t n = L.need.proj;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(uint32_t((n + 255) / 256)), dim3(256), 0, st, b->proj, n, 0ull);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipMemcpyAsync(b->meta, b->meta_host, table_bytes(S), hipMemcpyHostToDevice, st));
  const auto* dptr = static_cast<const uint64_t*>(b->meta);
  char* ybase = static_cast<char*>(b->y);
  // the first group's transform clears the job's counters (every correlation
  // kernel runs after all of the job's transforms)
  unsigned long long* zero = b->counter;
  for (const Group& g : L.groups) {
    const KernelSet& ks = *g.sp->ks;
    void* yg = ybase + g.y_off;
    const bfs_status rs = queue_segment_fft(*g.sp, g.count, dptr + g.first, nullptr, 0, yg, b->z, st, zero);
    zero = nullptr;
    if (rs != BFS_OK) return rs;
    if (p->fused) HIP_TRY(ks.permute_y(g.count, st, yg, ybase + g.yf_off));
  }
  return BFS_OK;
}

// The fused-synthesis fields of a correlation launch.
void set_fused_args(const bfs_plan* p, const SizePlan& sp, CorrArgs& c) {
  const auto* f0 = static_cast<const double*>(p->fparams);
  c.f0 = f0;
  c.fdot = f0 + p->K;
  c.len = reinterpret_cast<const uint32_t*>(f0 + 2ull * p->K);
  c.norm = p->fnorm;
  c.fs = p->fs;
  c.taper = p->taper;
  c.sym = p->sym;
  c.rows = sp.fused_rows;
}

// Queue the second part on cs: one fused correlation kernel per group, then
// (projection plans) the compaction of the projection keys.  With with_events,
// ev[1] / ev[2] are recorded as the first correlation kernel starts and the last
// one ends (by the launches themselves).
bfs_status enqueue_corr(bfs_plan* p, JobBuffers* b, const Layout& L, bool dense, void* rho, double* sigma,
                        hipStream_t cs, bool with_events, uint32_t first = 0, uint32_t count = 0) {
  if (!count) count = p->K;
  const uint32_t S = uint32_t(L.seg_len.size());
  const bool project = p->project && !dense;
  const auto* dptr = static_cast<const uint64_t*>(b->meta);
  const auto* dpoff = dptr + S;
  const auto* dlag0 = dpoff + S;
  const auto* dids = reinterpret_cast<const uint32_t*>(dlag0 + S + 1);
  char* ybase = static_cast<char*>(b->y);
  // ev[1] / ev[2] ride on the first and the last correlation launch
  if (with_events && L.groups.empty()) HIP_TRY(hipEventRecord(b->ev[1], cs));
  for (size_t gi = 0; gi < L.groups.size(); ++gi) {
    const Group& g = L.groups[gi];
    CorrArgs c{};
    c.ev_start = with_events && gi == 0 ? b->ev[1] : nullptr;
    c.ev_stop = with_events && gi + 1 == L.groups.size() ? b->ev[2] : nullptr;
    c.bank = p->fused ? nullptr
                      : static_cast<const char*>(g.sp->bank) + uint64_t(first) * g.sp->M * g.sp->ks->spec_size;
    c.y = ybase + (p->fused ? g.yf_off : g.y_off);
    c.seg_ids = dids + g.first;
    c.tw_u = g.sp->tw_u;
    c.tw1 = g.sp->tw1;
    c.tw2 = g.sp->tw2;
    c.K = count;
    c.tile = g.sp->tile;
    c.kappa = p->kappa;
    c.kappa_hi = p->kappa_hi;
    c.sigma = dense ? sigma : b->sigma;
    c.tails = b->tails;
    c.counter = b->counter;
    c.cap = dense ? 0 : p->cap;
    c.proj = project ? b->proj : nullptr;
    c.proj_off = project ? dpoff + g.first : nullptr;
    c.rho = rho;
    c.cus = p->cus;
    if (p->fused) {
      set_fused_args(p, *g.sp, c);
      if (first) {  // a slice of the bank: its templates' parameters
        c.f0 += first;
        c.fdot += first;
        c.len += first;
        c.norm += first;
      }
      HIP_TRY(g.sp->ks->corr_fused(dense, g.count, cs, c));
    } else {
      HIP_TRY(p->pairs ? g.sp->ks->corr_pair(dense, g.count, cs, c) : g.sp->ks->corr(dense, g.count, cs, c));
    }
  }
  if (with_events && L.groups.empty()) HIP_TRY(hipEventRecord(b->ev[2], cs));
  if (project) {
    const uint64_t n = L.need.proj;
    const uint32_t blocks = uint32_t(std::min<uint64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(project_compact_kernel, dim3(blocks), dim3(256), 0, cs, b->proj, n, b->plist, b->counter + 1,
                       n);
    HIP_TRY(hipGetLastError());
    if (p->delta > 0.0) {  // coincidences of the pairs' two projections
      uint32_t nmax = 0;
      for (uint32_t s = 0; s < S; ++s) nmax = std::max(nmax, L.seg_len[s]);
      const dim3 grid((nmax + 255) / 256, S / 2);
      hipLaunchKernelGGL(coinc_kernel, grid, dim3(256), 0, cs, b->proj, dlag0, p->f0_dev, p->delta, b->clist,
                         b->counter + 2, L.need.coinc);
      HIP_TRY(hipGetLastError());
    }
  }
  return BFS_OK;
}

// The whole job on one stream (graph capture, dense correlation).
// The job's counters and list heads to pinned host memory, on st after its
// kernels (publish_kernel).
bfs_status enqueue_publish(bfs_plan* p, JobBuffers* b, hipStream_t st) {
  const uint32_t tail_words = uint32_t(p->rec_bytes / 8);
  const PublishList lt{static_cast<const uint2*>(b->tails), static_cast<uint2*>(b->dev_pub_tails), b->pub_tails_cap,
                       tail_words};
  const PublishList lp{reinterpret_cast<const uint2*>(b->plist), static_cast<uint2*>(b->dev_pub_proj), b->pub_proj_cap,
                       2u};
  const PublishList lc{reinterpret_cast<const uint2*>(b->clist), static_cast<uint2*>(b->dev_pub_coinc),
                       b->pub_coinc_cap, uint32_t(sizeof(coinc_rec) / 8)};
  hipLaunchKernelGGL(publish_kernel, dim3(16), dim3(256), 0, st, b->counter,
                     static_cast<unsigned long long*>(b->dev_count_host), lt, lp, lc);
  HIP_TRY(hipGetLastError());
  return BFS_OK;
}

bfs_status enqueue_body(bfs_plan* p, JobBuffers* b, const Layout& L, bool dense, void* rho, double* sigma,
                        hipStream_t st, bool with_events, uint32_t first = 0, uint32_t count = 0) {
  bfs_status rs = enqueue_prep(p, b, L, dense, st);
  if (rs != BFS_OK) return rs;
  rs = enqueue_corr(p, b, L, dense, rho, sigma, st, with_events, first, count);
  if (rs != BFS_OK || dense) return rs;
  return enqueue_publish(p, b, st);
}

// The correlation stream paired with the caller's stream st (created on first
// use, non-blocking, default priority; destroyed with the plan).
constexpr size_t MAX_CORR_STREAMS = 16;
bfs_status corr_stream(bfs_plan* p, hipStream_t st, hipStream_t* out) {
  std::lock_guard<std::mutex> lk(p->stream_mu);
  for (const auto& e : p->corr_streams)
    if (e.first == st) {
      *out = e.second;
      return BFS_OK;
    }
  hipStream_t cs = nullptr;
  if (p->owned_streams.size() < MAX_CORR_STREAMS) {
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    p->owned_streams.push_back(cs);
  } else {
    cs = p->owned_streams[p->corr_streams.size() % MAX_CORR_STREAMS];
  }
  p->corr_streams.emplace_back(st, cs);
  *out = cs;
  return BFS_OK;
}

// Shape of a job as the graph cache sees it: the segment count and, per
// group, its length and count.  Everything else a replay needs (segment
// addresses, ids) flows through the pinned table the graph copies from.
std::vector<uint64_t> graph_key(const Layout& L) {
  std::vector<uint64_t> k{L.seg_len.size()};
  for (const Group& g : L.groups) k.push_back((uint64_t(g.sp->N) << 32) | g.count);
  return k;
}

// Capture the job body once per job-buffer set and shape on the plan's
// capture stream, then replay it on st.
bfs_status launch_graph(bfs_plan* p, JobBuffers* b, const Layout& L, hipStream_t st) {
  std::vector<uint64_t> key = graph_key(L);
  if (!b->gexec || b->gkey != key) {
    if (b->gexec) {
      (void)hipGraphExecDestroy(b->gexec);
      b->gexec = nullptr;
    }
    std::lock_guard<std::mutex> lk(p->capture_mu);
    hipStream_t cs = p->capture_stream;
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const bfs_status rs = enqueue_body(p, b, L, false, nullptr, nullptr, cs, false);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &g);
    if (rs != BFS_OK || ec != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      return BFS_ERR_HIP;
    }
    const hipError_t ei = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      b->gexec = nullptr;
      return BFS_ERR_HIP;
    }
    b->gkey = std::move(key);
  }
  HIP_TRY(hipEventRecord(b->ev[1], st));
  HIP_TRY(hipGraphLaunch(b->gexec, st));
  HIP_TRY(hipEventRecord(b->ev[2], st));
  return BFS_OK;
}

// Queue a job.  Tail and projection jobs outside graph plans split over two
// streams: the segment transforms on st, the correlation kernels on st's
// paired stream after them (ev[4]), so st is free for the next job's
// transforms while this job's correlations run; ev[b->done] marks the job
// done.  Graph plans and dense correlations keep the whole job on st.
// *done_stream is the stream that event was recorded on.
bfs_status queue_job(bfs_plan* p, JobBuffers* b, const Layout& L, bool dense, void* rho, double* sigma,
                     hipStream_t st, hipStream_t* done_stream, uint32_t first = 0, uint32_t count = 0) {
  *done_stream = st;
  HIP_TRY(hipEventRecord(b->ev[0], st));
  if (p->graph && !dense) {
    const bfs_status rs = launch_graph(p, b, L, st);
    if (rs != BFS_OK) return rs;
  } else if (dense) {
    const bfs_status rs = enqueue_body(p, b, L, dense, rho, sigma, st, true, first, count);
    if (rs != BFS_OK) return rs;
  } else {
    hipStream_t cs = nullptr;
    bfs_status rs = corr_stream(p, st, &cs);
    if (rs != BFS_OK) return rs;
    rs = enqueue_prep(p, b, L, false, st);
    if (rs != BFS_OK) return rs;
    HIP_TRY(hipEventRecord(b->ev[4], st));
    HIP_TRY(hipStreamWaitEvent(cs, b->ev[4], 0));
    *done_stream = cs;
    rs = enqueue_corr(p, b, L, false, nullptr, nullptr, cs, true);
    if (rs != BFS_OK) return rs;
    rs = enqueue_publish(p, b, cs);
    if (rs != BFS_OK) return rs;
  }
  b->done = dense ? 2 : 3;
  if (b->done == 3) HIP_TRY(hipEventRecord(b->ev[3], *done_stream));
  return BFS_OK;
}

// Fetches of at least DEVICE_SORT_MIN tails are ordered on the device.
constexpr uint64_t DEVICE_SORT_MIN = 1u << 15;

uint64_t sort_out_bytes(uint64_t n, size_t rec_bytes) { return (n * rec_bytes + 255) & ~uint64_t(255); }

// Make b's device sort area hold n records (grown to at most the tail
// capacity, kept with the buffers).  Its bytes count against the plan's HBM
// budget as part of the job; false (and the host sort) when they do not fit
// or the allocation fails.
bool ensure_sort(bfs_plan* p, JobBuffers* b, uint64_t n) {
  if (b->sorted && b->sort_cap >= n) return true;
  const uint64_t want = std::min<uint64_t>(p->cap, std::max<uint64_t>(n, 2 * b->sort_cap));
  const size_t work = tail_sort_work_bytes(want);
  if (!work) return false;
  const uint64_t bytes = sort_out_bytes(want, p->rec_bytes) + work;
  std::lock_guard<std::mutex> lk(p->mu);
  // the pooled buffer sets still hold device memory: count them, and give them back to the
  // device when the sort area fits only without them
  if (p->plan_bytes + p->live_job_bytes + p->pool_bytes - b->sort_bytes + bytes > p->budget) {
    if (p->plan_bytes + p->live_job_bytes - b->sort_bytes + bytes > p->budget) return false;
    for (auto* q : p->pool) free_job_buffers(q);
    p->pool.clear();
    p->pool_bytes = 0;
  }
  if (b->sorted) (void)hipFree(b->sorted);
  p->live_job_bytes -= b->sort_bytes;
  b->bytes -= b->sort_bytes;
  b->sorted = nullptr;
  b->sort_cap = 0;
  b->sort_bytes = 0;
  if (hipMalloc(&b->sorted, bytes) != hipSuccess) {
    b->sorted = nullptr;
    (void)hipGetLastError();
    return false;
  }
  b->sort_cap = want;
  b->sort_bytes = bytes;
  b->bytes += bytes;
  p->live_job_bytes += bytes;
  return true;
}

// Tails in (segment, template_id, lag) order.  The device writes them in
// whatever order the atomics hand out slots; sorting makes the result
// deterministic.  LSD radix sort (8-bit digits: 256 counters per pass, where
// 16-bit digits spend most of a small sort on clearing and scanning 65,536;
// passes whose digit is the same for every key are skipped) of the packed key
// segment << 48 | template_id << 17 | lag when every field fits (segments
// < 2^16, templates < 2^31, lags < 2^17), else a comparison sort.
template <typename R>
void sort_tails(R* t, uint64_t n) {
  auto less = [](const R& a, const R& c) {
    if (a.segment != c.segment) return a.segment < c.segment;
    if (a.template_id != c.template_id) return a.template_id < c.template_id;
    return a.lag < c.lag;
  };
  bool fits = n < (1ull << 32);
  for (uint64_t i = 0; i < n && fits; ++i)
    fits = t[i].segment < (1u << 16) && t[i].template_id < (1u << 31) && t[i].lag < (1u << 17);
  if (!fits || n < 4096) {
    std::sort(t, t + n, less);
    return;
  }
  std::vector<uint64_t> key(n), key2(n);
  std::vector<uint32_t> idx(n), idx2(n);
  for (uint64_t i = 0; i < n; ++i) {
    key[i] = (uint64_t(t[i].segment) << 48) | (uint64_t(t[i].template_id) << 17) | t[i].lag;
    idx[i] = uint32_t(i);
  }
  std::vector<uint64_t> count(1u << 8);
  for (int shift = 0; shift < 64; shift += 8) {
    std::fill(count.begin(), count.end(), 0);
    for (uint64_t i = 0; i < n; ++i) ++count[(key[i] >> shift) & 0xffu];
    if (*std::max_element(count.begin(), count.end()) == n) continue;  // one digit value: already ordered
    uint64_t sum = 0;
    for (auto& c : count) {
      const uint64_t v = c;
      c = sum;
      sum += v;
    }
    for (uint64_t i = 0; i < n; ++i) {
      const uint64_t d = (key[i] >> shift) & 0xffu;
      key2[count[d]] = key[i];
      idx2[count[d]++] = idx[i];
    }
    key.swap(key2);
    idx.swap(idx2);
  }
  std::vector<R> tmp(t, t + n);
  for (uint64_t i = 0; i < n; ++i) t[i] = tmp[idx[i]];
}

// The job's tails, ordered by (segment, template_id, lag), in the plan's
// record type in the job's pinned staging buffer: from 32,768 tails up
// sorted on the device (when the sort area fits the budget), else on the
// host.  *count: tails the kernels found; *on_dev: records the buffer holds.
template <typename R>
bfs_status sorted_tails(bfs_job* j, const R** recs, uint64_t* on_dev_out, unsigned long long* count_out) {
  bfs_plan* p = j->plan;
  JobBuffers* b = j->buf;
  HIP_TRY(hipEventSynchronize(b->ev[b->done]));
  const unsigned long long count = b->count_host[0];  // published at the job's end
  const uint64_t on_dev = std::min<uint64_t>(count, p->cap);
  if (on_dev < DEVICE_SORT_MIN && on_dev <= b->pub_tails_cap) {
    // the records are in host memory already: sort them where they are
    R* pub = static_cast<R*>(b->pub_tails);
    sort_tails(pub, on_dev);
    *recs = pub;
    *on_dev_out = on_dev;
    *count_out = count;
    return BFS_OK;
  }
  if (on_dev > b->tails_host_cap) {
    if (b->tails_host) (void)hipHostFree(b->tails_host);
    b->tails_host = nullptr;
    b->tails_host_cap = 0;
    const uint64_t want = std::min<uint64_t>(p->cap, std::max<uint64_t>(on_dev, 2 * on_dev));
    if (hipHostMalloc(&b->tails_host, want * sizeof(R), hipHostMallocDefault) != hipSuccess) {
      b->tails_host = nullptr;
      (void)hipGetLastError();
      return BFS_ERR_OUT_OF_MEMORY;
    }
    b->tails_host_cap = want;
  }
  R* tmp = static_cast<R*>(b->tails_host);
  bool sorted = false;
  if (on_dev >= DEVICE_SORT_MIN && p->K < (1u << 31) && p->n_max <= (1u << 17) && ensure_sort(p, b, on_dev)) {
    // order on the device, then one copy of the sorted records
    const uint32_t end_bit = j->S > 1 ? 48u + uint32_t(32 - __builtin_clz(j->S - 1)) : 48u;
    char* work = static_cast<char*>(b->sorted) + sort_out_bytes(b->sort_cap, sizeof(R));
    if (tail_sort(b->tails, sizeof(R), on_dev, end_bit, work, b->sort_bytes - sort_out_bytes(b->sort_cap, sizeof(R)),
                  b->sorted, p->copy_stream) == hipSuccess) {
      HIP_TRY(hipMemcpyAsync(tmp, b->sorted, on_dev * sizeof(R), hipMemcpyDeviceToHost, p->copy_stream));
      HIP_TRY(hipStreamSynchronize(p->copy_stream));
      sorted = true;
    } else {
      (void)hipGetLastError();
      HIP_TRY(hipStreamSynchronize(p->copy_stream));
    }
  }
  if (!sorted) {
    if (on_dev) {
      HIP_TRY(hipMemcpyAsync(tmp, b->tails, on_dev * sizeof(R), hipMemcpyDeviceToHost, p->copy_stream));
      HIP_TRY(hipStreamSynchronize(p->copy_stream));
    }
    sort_tails(tmp, on_dev);
  }
  *recs = tmp;
  *on_dev_out = on_dev;
  *count_out = count;
  return BFS_OK;
}

// One record of the plan's type as the caller's record type (the value of rho
// rounded to float for bfs_tail, exact for bfs_tail64).
template <typename Out, typename R>
Out as_record(const R& r) {
  Out o{};
  o.segment = r.segment;
  o.template_id = r.template_id;
  o.lag = r.lag;
  o.rho = decltype(o.rho)(r.rho);
  return o;
}

template <typename Out>
bfs_status fetch_tails_as(bfs_job* j, Out* out_host, uint64_t capacity, uint64_t* n_written, uint64_t* n_total) {
  if (!j || !n_written || !n_total || (capacity > 0 && !out_host)) return BFS_ERR_INVALID_ARG;
  bfs_plan* p = j->plan;
  if (p->project) return BFS_ERR_INVALID_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return BFS_ERR_HIP;
  uint64_t on_dev = 0, nw = 0;
  unsigned long long count = 0;
  bfs_status st;
  auto copy = [&](const auto* r) {
    using R = std::remove_cv_t<std::remove_pointer_t<decltype(r)>>;
    nw = std::min<uint64_t>(on_dev, capacity);
    if (sizeof(R) == sizeof(Out)) {  // the caller's record is the plan's (same layout)
      if (nw) std::memcpy(out_host, r, nw * sizeof(Out));
    } else {
      for (uint64_t i = 0; i < nw; ++i) out_host[i] = as_record<Out>(r[i]);
    }
  };
  if (p->rec_bytes == sizeof(tail_rec64)) {
    const tail_rec64* r = nullptr;
    st = sorted_tails(j, &r, &on_dev, &count);
    if (st == BFS_OK) copy(r);
  } else {
    const tail_rec* r = nullptr;
    st = sorted_tails(j, &r, &on_dev, &count);
    if (st == BFS_OK) copy(r);
  }
  if (st != BFS_OK) return st;
  *n_written = nw;
  *n_total = count;
  return (count > nw) ? BFS_ERR_TAIL_OVERFLOW : BFS_OK;
}

// ------------------------------------------------------------ no-allocation scratch --
// The segment spectra (and the split length's transform scratch) of
// bfsearch_filter_noalloc live in this array, one copy per device, held until
// the process ends.  Host code never passes the array's name to a kernel: its
// device address on each device comes from hipGetSymbolAddress (scratch_address)
// and only that address is used.
constexpr uint64_t NOALLOC_SCRATCH_BYTES = BFS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device ordinal; null until looked up

// The device address of `scratch` on `device`, which must be the current
// device; looked up once per device.
bfs_status scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0) return BFS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (size_t(device) < g_scratch_ptr.size() && g_scratch_ptr[size_t(device)]) {
    *out = g_scratch_ptr[size_t(device)];
    return BFS_OK;
  }
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return BFS_ERR_HIP;
  }
  if (g_scratch_ptr.size() <= size_t(device)) g_scratch_ptr.resize(size_t(device) + 1, nullptr);
  g_scratch_ptr[size_t(device)] = ptr;
  *out = ptr;
  return BFS_OK;
}

}  // namespace

extern "C" {

const char* bfsearch_status_string(bfs_status s) {
  switch (s) {
    case BFS_OK: return "ok";
    case BFS_ERR_INVALID_ARG: return "invalid argument";
    case BFS_ERR_OUT_OF_MEMORY: return "out of device memory or HBM budget";
    case BFS_ERR_HIP: return "HIP runtime error";
    case BFS_ERR_TAIL_OVERFLOW: return "tail buffer overflow";
    case BFS_ERR_UNSUPPORTED: return "unsupported configuration";
    case BFS_ERR_SCRATCH_LIMIT: return "request exceeds the no-allocation scratch area";
  }
  return "unknown status";
}

bfs_status bfsearch_plan(const bfs_plan_desc* d, bfs_plan** out) {
  if (!out) return BFS_ERR_INVALID_ARG;
  *out = nullptr;
  const bfs_status v = validate(d);
  if (v != BFS_OK) return v;
  auto* p = new (std::nothrow) bfs_plan();
  if (!p) return BFS_ERR_OUT_OF_MEMORY;
  p->device = d->device;
  p->n_max = d->n;
  p->n_min = n_min_of(d);
  p->K = d->explicit_templates ? d->n_explicit : d->n_f0 * d->n_fdot;
  p->prec = d->precision;
  p->kappa = d->kappa;
  p->kappa_hi = d->kappa_hi;
  p->cap = d->tail_capacity;
  p->rec_bytes = d->precision == BFS_FP64 ? sizeof(tail_rec64) : sizeof(tail_rec);
  size_plans(p, d, (d->flags & BFS_PLAN_FUSED) != 0);
  p->pairs = (d->flags & BFS_PLAN_PAIRS) != 0;
  p->delta = d->coinc_delta_hz;
  if (p->delta > 0.0) p->plan_bytes += uint64_t(p->K) * sizeof(double);
  if (hipSetDevice(d->device) != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return BFS_ERR_HIP;
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    delete p;
    return BFS_ERR_HIP;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d->device) != hipSuccess || cus < 0) {
    (void)hipGetLastError();
    cus = 0;
  }
  p->cus = uint32_t(cus);
  // the no-allocation entry point's scratch area on this device (looked up once per
  // device; a failed lookup only disables that entry point)
  if (scratch_address(d->device, &p->scratch) != BFS_OK) p->scratch = nullptr;
  p->budget = d->hbm_budget_bytes ? std::min<uint64_t>(d->hbm_budget_bytes, free_b) : free_b;
  // a resident bank that does not fit falls back to fused synthesis where that serves the plan
  if (p->plan_bytes > p->budget && !p->fused && fused_possible(d)) size_plans(p, d, true);
  if (p->plan_bytes > p->budget) {
    free_plan(p);
    return BFS_ERR_OUT_OF_MEMORY;
  }
  p->graph = (d->flags & BFS_PLAN_GRAPH) != 0;
  p->project = (d->flags & BFS_PLAN_PROJECT) != 0;
  if (hipStreamCreateWithFlags(&p->copy_stream, hipStreamNonBlocking) != hipSuccess ||
      (p->graph && hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) != hipSuccess)) {
    free_plan(p);
    return BFS_ERR_HIP;
  }
  bfs_status st = BFS_OK;
  for (SizePlan& sp : p->sizes) {
    if (!p->fused) st = alloc_checked(&sp.bank, sp.bank_bytes);
    if (st == BFS_OK) st = alloc_checked(&sp.tables, sp.tab_bytes);
    if (st == BFS_OK) st = set_tables(sp, sp.ks);
    if (st == BFS_OK && sp.sub) st = set_sub_tables(sp);
    if (st != BFS_OK) break;
  }
  if (st == BFS_OK) st = p->fused ? build_fused(p, d) : build_banks(p, d);
  if (st == BFS_OK && p->delta > 0.0) {  // initial frequency per template, for the coincidence window
    std::vector<double> f0(p->K);
    for (uint32_t j = 0; j < p->K; ++j) f0[j] = linspace_at(d->f0_lo, d->f0_hi, d->n_f0, j / d->n_fdot);
    st = alloc_checked(reinterpret_cast<void**>(&p->f0_dev), uint64_t(p->K) * sizeof(double));
    if (st == BFS_OK && hipMemcpy(p->f0_dev, f0.data(), f0.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      st = BFS_ERR_HIP;
  }
  if (st == BFS_OK && (d->flags & BFS_PLAN_AUTOTUNE) && !d->candidate && !d->tile && !p->fused)
    for (SizePlan& sp : p->sizes)
      if (st == BFS_OK) st = tune_size(p, sp);
  if (st != BFS_OK) {
    free_plan(p);
    return st;
  }
  *out = p;
  return BFS_OK;
}

bfs_status bfsearch_plan_get_info(const bfs_plan* p, bfs_plan_info* out) {
  if (!p || !out) return BFS_ERR_INVALID_ARG;
  out->n = p->n_max;
  out->m = p->n_max / 2;
  out->k = p->K;
  out->threads_per_correlation = uint32_t(p->sizes.back().ks->NT);
  out->bank_bytes = p->bank_bytes;
  out->plan_bytes = p->plan_bytes;
  out->precision = uint32_t(p->prec);
  out->n_min = p->n_min;
  {
    std::lock_guard<std::mutex> lk(const_cast<bfs_plan*>(p)->mu);
    out->held_bytes = p->plan_bytes + p->live_job_bytes + p->pool_bytes;
  }
  return BFS_OK;
}

bfs_status bfsearch_plan_kernel_info(const bfs_plan* p, uint32_t n, bfs_kernel_info* out) {
  if (!p || !out) return BFS_ERR_INVALID_ARG;
  const SizePlan* sp = size_plan(p, n ? n : p->n_max);
  if (!sp) return BFS_ERR_INVALID_ARG;
  std::memset(out, 0, sizeof(*out));
  out->n = sp->N;
  out->r1 = uint32_t(sp->ks->R1);
  out->r2 = uint32_t(sp->ks->R2);
  out->r3 = uint32_t(sp->ks->R3);
  out->threads = uint32_t(sp->ks->NT);
  out->load_group = uint32_t(sp->ks->G);
  out->split = uint32_t(sp->ks->split);
  out->candidate = uint32_t(sp->cand);
  out->n_candidates = uint32_t(sp->n_cand);
  for (int i = 0; i < MAX_CANDIDATES && i < 8; ++i) out->tuned_us[i] = sp->tuned_us[i];
  out->tile = sp->tile;
  for (int i = 0; i < N_TILES; ++i) out->tile_us[i] = sp->tile_us[i];
  out->fused = p->fused ? 1u : 0u;
  out->loop = uint32_t(sp->ks->loop);
  out->fused_rows = sp->fused_rows;
  return BFS_OK;
}

bfs_status bfsearch_filter(bfs_plan* p, const void* y_dev, const uint64_t* seg_offsets, const uint32_t* seg_lengths,
                           uint32_t S, void* hip_stream, bfs_job** out) {
  if (!out) return BFS_ERR_INVALID_ARG;
  *out = nullptr;
  if (!p || !y_dev || S < 1 || S > 65535) return BFS_ERR_INVALID_ARG;
  Layout L;
  bfs_status rs = make_layout(p, seg_lengths, S, L);
  if (rs != BFS_OK) return rs;
  auto* j = new (std::nothrow) bfs_job();
  if (!j) return BFS_ERR_OUT_OF_MEMORY;
  if (hipSetDevice(p->device) != hipSuccess) {
    delete j;
    return BFS_ERR_HIP;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  JobBuffers* b = nullptr;
  rs = get_job_buffers(p, L.need, &b);
  if (rs != BFS_OK) {
    delete j;
    return rs;
  }
  stage_table(p, y_dev, seg_offsets, L, b->meta_host);
  hipStream_t done_st = st;
  rs = queue_job(p, b, L, false, nullptr, nullptr, st, &done_st);
  if (rs != BFS_OK) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamSynchronize(done_st);
    put_job_buffers(p, b);
    delete j;
    return rs;
  }
  j->plan = p;
  j->buf = b;
  j->stream = st;
  j->S = S;
  j->groups = std::move(L.groups);
  j->seg_len = std::move(L.seg_len);
  *out = j;
  return BFS_OK;
}

bfs_status bfsearch_filter_noalloc(bfs_plan* p, const void* y_dev, uint32_t seg_len, uint32_t S, void* tails_dev,
                                   uint64_t tail_capacity, uint64_t* count_dev, double* sigma_dev, void* hip_stream) {
  if (!p || !y_dev || !count_dev || S < 1 || S > 65535 || (tail_capacity && !tails_dev)) return BFS_ERR_INVALID_ARG;
  if (p->project) return BFS_ERR_INVALID_ARG;
  if (!seg_len) seg_len = p->n_max;
  const SizePlan* sp = size_plan(p, seg_len);
  if (!sp) return BFS_ERR_INVALID_ARG;
  if (p->pairs && (S & 1u)) return BFS_ERR_INVALID_ARG;
  const KernelSet& ks = *sp->ks;
  // segment spectra, then a scratch of the same size: the transform's (split and joined
  // segment transforms) and the fused-layout copy (fused plans) in turn
  const uint64_t spec_bytes = uint64_t(S) * sp->M * 2 * ks.real_size;
  const uint64_t y_bytes = (spec_bytes + 255) & ~uint64_t(255);
  const bool joined = ks.join && sp->sub;
  const uint64_t z_bytes = (ks.split || p->fused || joined) ? spec_bytes : 0;
  if (y_bytes + z_bytes > NOALLOC_SCRATCH_BYTES) return BFS_ERR_SCRATCH_LIMIT;
  if (!p->scratch) return BFS_ERR_HIP;
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != p->device) HIP_TRY(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  char* y = static_cast<char*>(p->scratch);
  void* z = (ks.split || p->fused || joined) ? y + y_bytes : nullptr;
  auto* counter = reinterpret_cast<unsigned long long*>(count_dev);
  // the count starts at zero (a fill kernel, so the call can be captured in a graph)
  hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(64), 0, st, counter, uint64_t(1), 0ull);
  HIP_TRY(hipGetLastError());
  // segments packed back to back
  const bfs_status rs = queue_segment_fft(*sp, S, nullptr, y_dev, seg_len, y, z, st);
  if (rs != BFS_OK) return rs;
  if (p->fused) HIP_TRY(ks.permute_y(S, st, y, z));
  CorrArgs c{};
  c.bank = sp->bank;
  c.y = p->fused ? z : y;
  c.seg_ids = nullptr;  // row r is segment r
  c.tw_u = sp->tw_u;
  c.tw1 = sp->tw1;
  c.tw2 = sp->tw2;
  c.K = p->K;
  c.tile = sp->tile;
  c.kappa = p->kappa;
  c.kappa_hi = p->kappa_hi;
  c.sigma = sigma_dev;
  c.tails = tails_dev;
  c.counter = counter;
  c.cap = tail_capacity;
  c.cus = p->cus;
  if (p->fused) {
    set_fused_args(p, *sp, c);
    HIP_TRY(ks.corr_fused(false, S, st, c));
  } else {
    HIP_TRY(p->pairs ? ks.corr_pair(false, S, st, c) : ks.corr(false, S, st, c));
  }
  return BFS_OK;
}

bfs_status bfsearch_fetch_tails(bfs_job* j, bfs_tail* out_host, uint64_t capacity, uint64_t* n_written,
                                uint64_t* n_total) {
  return fetch_tails_as(j, out_host, capacity, n_written, n_total);
}

bfs_status bfsearch_fetch_tails64(bfs_job* j, bfs_tail64* out_host, uint64_t capacity, uint64_t* n_written,
                                  uint64_t* n_total) {
  return fetch_tails_as(j, out_host, capacity, n_written, n_total);
}

bfs_status bfsearch_fetch_projection(bfs_job* j, bfs_peak* out_host, uint64_t capacity, uint64_t* n_written,
                                     uint64_t* n_total) {
  if (!j || !n_written || !n_total || (capacity > 0 && !out_host)) return BFS_ERR_INVALID_ARG;
  bfs_plan* p = j->plan;
  if (!p->project) return BFS_ERR_INVALID_ARG;
  JobBuffers* b = j->buf;
  if (hipSetDevice(p->device) != hipSuccess) return BFS_ERR_HIP;
  HIP_TRY(hipEventSynchronize(b->ev[b->done]));
  const unsigned long long count = b->count_host[1];  // <= the number of lags, the list's size
  std::vector<unsigned long long> list(2 * count);
  if (count && count <= b->pub_proj_cap) {
    std::memcpy(list.data(), b->pub_proj, 2 * count * sizeof(unsigned long long));
  } else if (count) {
    HIP_TRY(hipMemcpyAsync(list.data(), b->plist, 2 * count * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           p->copy_stream));
    HIP_TRY(hipStreamSynchronize(p->copy_stream));
  }
  // global lag index -> (segment, lag): segments back to back in the caller's order
  std::vector<uint64_t> lag0(j->S + 1, 0);
  for (uint32_t s = 0; s < j->S; ++s) lag0[s + 1] = lag0[s] + j->seg_len[s];
  std::vector<bfs_peak> peaks(count);
  for (uint64_t i = 0; i < count; ++i) {
    const uint64_t idx = list[2 * i];
    const unsigned long long key = list[2 * i + 1];
    const uint32_t s = uint32_t(std::upper_bound(lag0.begin(), lag0.end(), idx) - lag0.begin() - 1);
    const uint32_t lo = uint32_t(key & 0xffffffffull);
    const uint32_t bits = uint32_t(key >> 32);
    float snr;
    std::memcpy(&snr, &bits, sizeof(snr));
    peaks[i].segment = s;
    peaks[i].lag = uint32_t(idx - lag0[s]);
    peaks[i].template_id = 0x7fffffffu - (lo >> 1);
    peaks[i].snr = (lo & 1u) ? -snr : snr;
  }
  std::sort(peaks.begin(), peaks.end(), [](const bfs_peak& a, const bfs_peak& c) {
    return a.segment != c.segment ? a.segment < c.segment : a.lag < c.lag;
  });
  const uint64_t nw = std::min<uint64_t>(count, capacity);
  if (nw) std::memcpy(out_host, peaks.data(), nw * sizeof(bfs_peak));
  *n_written = nw;
  *n_total = count;
  return (count > nw) ? BFS_ERR_TAIL_OVERFLOW : BFS_OK;
}

bfs_status bfsearch_fetch_coincidences(bfs_job* j, bfs_coinc* out_host, uint64_t capacity, uint64_t* n_written,
                                       uint64_t* n_total) {
  if (!j || !n_written || !n_total || (capacity > 0 && !out_host)) return BFS_ERR_INVALID_ARG;
  bfs_plan* p = j->plan;
  if (!(p->delta > 0.0)) return BFS_ERR_INVALID_ARG;
  JobBuffers* b = j->buf;
  if (hipSetDevice(p->device) != hipSuccess) return BFS_ERR_HIP;
  HIP_TRY(hipEventSynchronize(b->ev[b->done]));
  const unsigned long long count = b->count_host[2];  // <= the pairs' lags, the list's size
  std::vector<coinc_rec> list(count);
  if (count && count <= b->pub_coinc_cap) {
    std::memcpy(list.data(), b->pub_coinc, count * sizeof(coinc_rec));
  } else if (count) {
    HIP_TRY(hipMemcpyAsync(list.data(), b->clist, count * sizeof(coinc_rec), hipMemcpyDeviceToHost, p->copy_stream));
    HIP_TRY(hipStreamSynchronize(p->copy_stream));
  }
  std::sort(list.begin(), list.end(), [](const coinc_rec& a, const coinc_rec& c) {
    return a.pair != c.pair ? a.pair < c.pair : a.lag < c.lag;
  });
  const uint64_t nw = std::min<uint64_t>(count, capacity);
  for (uint64_t i = 0; i < nw; ++i)
    out_host[i] = bfs_coinc{list[i].pair, list[i].lag, list[i].template_a, list[i].template_b, list[i].snr_a,
                            list[i].snr_b};
  *n_written = nw;
  *n_total = count;
  return (count > nw) ? BFS_ERR_TAIL_OVERFLOW : BFS_OK;
}

bfs_status bfsearch_fetch_sigma(bfs_job* j, double* out_host) {
  if (!j || !out_host) return BFS_ERR_INVALID_ARG;
  bfs_plan* p = j->plan;
  if (hipSetDevice(p->device) != hipSuccess) return BFS_ERR_HIP;
  HIP_TRY(hipStreamWaitEvent(p->copy_stream, j->buf->ev[j->buf->done], 0));
  HIP_TRY(hipMemcpyAsync(out_host, j->buf->sigma, uint64_t(j->S) * p->K * sizeof(double), hipMemcpyDeviceToHost,
                         p->copy_stream));
  HIP_TRY(hipStreamSynchronize(p->copy_stream));
  return BFS_OK;
}

bfs_status bfsearch_job_timing(bfs_job* j, float* corr_ms, float* total_ms) {
  if (!j || !corr_ms || !total_ms) return BFS_ERR_INVALID_ARG;
  HIP_TRY(hipEventSynchronize(j->buf->ev[j->buf->done]));
  HIP_TRY(hipEventElapsedTime(corr_ms, j->buf->ev[1], j->buf->ev[2]));
  HIP_TRY(hipEventElapsedTime(total_ms, j->buf->ev[0], j->buf->ev[j->buf->done]));
  return BFS_OK;
}

bfs_status bfsearch_job_poll(bfs_job* j, int* done) {
  if (!j || !done) return BFS_ERR_INVALID_ARG;
  const hipError_t e = hipEventQuery(j->buf->ev[j->buf->done]);
  if (e == hipSuccess) {
    *done = 1;
    return BFS_OK;
  }
  if (e == hipErrorNotReady) {
    (void)hipGetLastError();
    *done = 0;
    return BFS_OK;
  }
  return BFS_ERR_HIP;
}

bfs_status bfsearch_plan_job_bytes(const bfs_plan* p, const uint32_t* seg_lengths, uint32_t S, uint64_t* bytes) {
  if (!p || !bytes || S < 1 || S > 65535) return BFS_ERR_INVALID_ARG;
  Layout L;
  const bfs_status rs = make_layout(p, seg_lengths, S, L);
  if (rs != BFS_OK) return rs;
  *bytes = need_bytes(L.need, p->cap, p->rec_bytes);
  return BFS_OK;
}

bfs_status bfsearch_job_release(bfs_job* j) {
  if (!j) return BFS_ERR_INVALID_ARG;
  // buffers may be reused by the next filter call: wait for this job's kernels
  (void)hipEventSynchronize(j->buf->ev[j->buf->done]);
  put_job_buffers(j->plan, j->buf);
  delete j;
  return BFS_OK;
}

bfs_status bfsearch_destroy(bfs_plan* p) {
  if (!p) return BFS_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->live_jobs) return BFS_ERR_INVALID_ARG;
  }
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  free_plan(p);
  return BFS_OK;
}

bfs_status bfsearch_correlate_dense_range(bfs_plan* p, const void* y_dev, uint32_t seg_len, uint32_t S,
                                          uint32_t first, uint32_t count, void* rho_dev, double* sigma_dev,
                                          void* hip_stream) {
  if (!p || !y_dev || !rho_dev || S < 1 || S > 65535) return BFS_ERR_INVALID_ARG;
  if (count < 1 || uint64_t(first) + count > p->K) return BFS_ERR_INVALID_ARG;
  if (!seg_len) seg_len = p->n_max;
  if (!size_plan(p, seg_len)) return BFS_ERR_INVALID_ARG;
  std::vector<uint32_t> lens(S, seg_len);
  Layout L;
  bfs_status rs = make_layout(p, lens.data(), S, L);
  if (rs != BFS_OK) return rs;
  L.need.sigma = uint64_t(S) * count;
  if (hipSetDevice(p->device) != hipSuccess) return BFS_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  JobBuffers* b = nullptr;
  rs = get_job_buffers(p, L.need, &b);
  if (rs != BFS_OK) return rs;
  stage_table(p, y_dev, nullptr, L, b->meta_host);
  hipStream_t done_st = st;
  rs = queue_job(p, b, L, true, rho_dev, sigma_dev, st, &done_st, first, count);
  // the buffers go back to the pool only after the queued kernels finish
  (void)hipStreamSynchronize(st);
  put_job_buffers(p, b);
  return rs;
}

bfs_status bfsearch_correlate_dense(bfs_plan* p, const void* y_dev, uint32_t seg_len, uint32_t S, void* rho_dev,
                                    double* sigma_dev, void* hip_stream) {
  if (!p) return BFS_ERR_INVALID_ARG;
  return bfsearch_correlate_dense_range(p, y_dev, seg_len, S, 0, p->K, rho_dev, sigma_dev, hip_stream);
}

bfs_status bfsearch_plan_spectra(const bfs_plan* p, uint32_t n, uint32_t first, uint32_t count, double* out_dev,
                                 void* hip_stream) {
  if (!p || !out_dev || count < 1 || uint64_t(first) + count > p->K || count > 65535) return BFS_ERR_INVALID_ARG;
  const SizePlan* sp = size_plan(p, n ? n : p->n_max);
  if (!sp) return BFS_ERR_INVALID_ARG;
  if (p->fused) return BFS_ERR_UNSUPPORTED;  // no resident bank
  if (hipSetDevice(p->device) != hipSuccess) return BFS_ERR_HIP;
  HIP_TRY(sp->ks->export_bank(count, static_cast<hipStream_t>(hip_stream), sp->bank, out_dev, first));
  return BFS_OK;
}

bfs_status bfsearch_job_spectra(const bfs_job* j, double* out_dev) {
  if (!j || !out_dev) return BFS_ERR_INVALID_ARG;
  if (hipSetDevice(j->plan->device) != hipSuccess) return BFS_ERR_HIP;
  // output in global segment order: segment s at sum_{s' < s} (N_s'/2 + 1) complex values
  std::vector<uint64_t> out_off(j->S);
  uint64_t acc = 0;
  for (uint32_t s = 0; s < j->S; ++s) {
    out_off[s] = acc;
    acc += 2ull * (j->seg_len[s] / 2 + 1);
  }
  const char* ybase = static_cast<const char*>(j->buf->y);
  for (const Group& g : j->groups) {
    const KernelSet& ks = *g.sp->ks;
    uint32_t k = 0;
    for (uint32_t s = 0; s < j->S; ++s) {
      if (j->seg_len[s] != g.sp->N) continue;
      const char* row = ybase + g.y_off + uint64_t(k) * g.sp->M * 2 * ks.real_size;
      HIP_TRY(ks.export_y(1, j->stream, row, out_dev + out_off[s]));
      ++k;
    }
  }
  return BFS_OK;
}

}  // extern "C"
