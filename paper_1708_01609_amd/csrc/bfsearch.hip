// C ABI and host runtime of the matched-filter library (see include/bfsearch.h).
//
// A plan owns the resident template bank (spectra of every template, built
// on the device at plan time) and the FFT twiddle tables.  A job owns the
// per-call buffers (segment spectra, sigma, tail buffer, tail counter) which
// return to a per-plan pool on release, so steady-state filter calls do not
// allocate.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "bfsearch.h"
#include "bfs_kernels.h"

using namespace bfs;

static_assert(sizeof(tail_rec) == sizeof(bfs_tail), "tail record layout");

namespace {

// ---------------------------------------------------------------- kernels --
// Kernel configuration per (real type, M = N/2): radices R1*R2*R3 = M and
// threads per workgroup.
template <typename T, int M>
struct CfgFor;
template <> struct CfgFor<float, 512> { using F = Fft3<float, 8, 8, 8, 64>; };
template <> struct CfgFor<float, 1024> { using F = Fft3<float, 4, 16, 16, 64>; };
template <> struct CfgFor<float, 2048> { using F = Fft3<float, 8, 16, 16, 128>; };
template <> struct CfgFor<float, 4096> { using F = Fft3<float, 16, 16, 16, 256>; };
template <> struct CfgFor<float, 8192> { using F = Fft3<float, 8, 32, 32, 256>; };
template <> struct CfgFor<float, 16384> { using F = Fft3<float, 16, 32, 32, 512>; };
template <> struct CfgFor<float, 32768> { using F = Fft3<float, 32, 32, 32, 1024>; };
template <> struct CfgFor<double, 512> { using F = Fft3<double, 8, 8, 8, 64>; };
template <> struct CfgFor<double, 1024> { using F = Fft3<double, 4, 16, 16, 64>; };
template <> struct CfgFor<double, 2048> { using F = Fft3<double, 8, 16, 16, 128>; };
template <> struct CfgFor<double, 4096> { using F = Fft3<double, 16, 16, 16, 256>; };

struct FwdArgs {
  const void* src;
  uint64_t src_stride;
  uint32_t src_len;
  const double* f0;
  const double* fdot;
  const uint32_t* len;
  double fs;
  int taper;
  uint32_t first;
  const void* tw1;
  const void* tw2;
  void* out;
  double* inv_norm;
};

struct CorrArgs {
  const void* bank;
  const void* y;
  const void* tw_u;
  const void* tw1;
  const void* tw2;
  uint32_t K;
  double kappa;
  double* sigma;
  tail_rec* tails;
  unsigned long long* counter;
  uint64_t cap;
  void* rho;
};

struct KernelSet {
  int R1, R2, R3, NT, M;
  size_t real_size;  // sizeof(T)
  size_t spec_size;  // bytes of one stored template spectrum element
  hipError_t (*fwd)(int src, uint32_t batch, hipStream_t st, const FwdArgs& a);
  hipError_t (*unpack_bank)(uint32_t batch, hipStream_t st, const void* Z, void* out, const double* scale,
                            const void* tw_u, uint64_t row_off);
  hipError_t (*unpack_y)(uint32_t batch, hipStream_t st, void* Z, const void* tw_u);
  hipError_t (*corr)(bool dense, uint32_t S, hipStream_t st, const CorrArgs& a);
  hipError_t (*export_bank)(uint32_t count, hipStream_t st, const void* bank, double* out, uint64_t first);
  hipError_t (*export_y)(uint32_t count, hipStream_t st, const void* y, double* out);
};

template <typename T, typename TW, class F>
struct Impl {
  static hipError_t fwd(int src, uint32_t batch, hipStream_t st, const FwdArgs& a) {
    const dim3 grid(batch), block(F::NT);
    const auto* t1 = static_cast<const cx<T>*>(a.tw1);
    const auto* t2 = static_cast<const cx<T>*>(a.tw2);
    auto* out = static_cast<cx<T>*>(a.out);
    if (src == SRC_SAMPLES)
      hipLaunchKernelGGL((fwd_fft_kernel<T, F, SRC_SAMPLES>), grid, block, 0, st, a.src, a.src_stride, a.src_len,
                         a.f0, a.fdot, a.len, a.fs, a.taper, a.first, t1, t2, out, a.inv_norm);
    else if (src == SRC_CHIRP)
      hipLaunchKernelGGL((fwd_fft_kernel<T, F, SRC_CHIRP>), grid, block, 0, st, a.src, a.src_stride, a.src_len,
                         a.f0, a.fdot, a.len, a.fs, a.taper, a.first, t1, t2, out, a.inv_norm);
    else
      hipLaunchKernelGGL((fwd_fft_kernel<T, F, SRC_EXPLICIT>), grid, block, 0, st, a.src, a.src_stride, a.src_len,
                         a.f0, a.fdot, a.len, a.fs, a.taper, a.first, t1, t2, out, a.inv_norm);
    return hipGetLastError();
  }
  static hipError_t unpack_bank(uint32_t batch, hipStream_t st, const void* Z, void* out, const double* scale,
                                const void* tw_u, uint64_t row_off) {
    const dim3 grid((F::M / 2 + 1 + 255) / 256, batch);
    hipLaunchKernelGGL((rfft_unpack_kernel<T, TW>), grid, dim3(256), 0, st, static_cast<const cx<T>*>(Z),
                       static_cast<TW*>(out), scale, static_cast<const cx<T>*>(tw_u), uint32_t(F::M), row_off);
    return hipGetLastError();
  }
  static hipError_t unpack_y(uint32_t batch, hipStream_t st, void* Z, const void* tw_u) {
    const dim3 grid((F::M / 2 + 1 + 255) / 256, batch);
    hipLaunchKernelGGL((rfft_unpack_kernel<T, cx<T>>), grid, dim3(256), 0, st, static_cast<const cx<T>*>(Z),
                       static_cast<cx<T>*>(Z), static_cast<const double*>(nullptr),
                       static_cast<const cx<T>*>(tw_u), uint32_t(F::M), uint64_t(0));
    return hipGetLastError();
  }
  static hipError_t corr(bool dense, uint32_t S, hipStream_t st, const CorrArgs& a) {
    const dim3 grid(a.K, S), block(F::NT);
    const auto* bank = static_cast<const TW*>(a.bank);
    const auto* y = static_cast<const cx<T>*>(a.y);
    const auto* tu = static_cast<const cx<T>*>(a.tw_u);
    const auto* t1 = static_cast<const cx<T>*>(a.tw1);
    const auto* t2 = static_cast<const cx<T>*>(a.tw2);
    if (dense)
      hipLaunchKernelGGL((corr_kernel<T, TW, F, true>), grid, block, 0, st, bank, y, tu, t1, t2, a.K, a.kappa,
                         a.sigma, a.tails, a.counter, a.cap, static_cast<T*>(a.rho));
    else
      hipLaunchKernelGGL((corr_kernel<T, TW, F, false>), grid, block, 0, st, bank, y, tu, t1, t2, a.K, a.kappa,
                         a.sigma, a.tails, a.counter, a.cap, static_cast<T*>(nullptr));
    return hipGetLastError();
  }
  static hipError_t export_bank(uint32_t count, hipStream_t st, const void* bank, double* out, uint64_t first) {
    const dim3 grid((F::M + 1 + 255) / 256, count);
    hipLaunchKernelGGL((spectrum_export_kernel<T, TW>), grid, dim3(256), 0, st, static_cast<const TW*>(bank), out,
                       uint32_t(F::M), first);
    return hipGetLastError();
  }
  static hipError_t export_y(uint32_t count, hipStream_t st, const void* y, double* out) {
    const dim3 grid((F::M + 1 + 255) / 256, count);
    hipLaunchKernelGGL((spectrum_export_kernel<T, cx<T>>), grid, dim3(256), 0, st, static_cast<const cx<T>*>(y),
                       out, uint32_t(F::M), uint64_t(0));
    return hipGetLastError();
  }
  static const KernelSet* get() {
    static const KernelSet ks = {F::R1, F::R2, F::R3, F::NT, F::M, sizeof(T), sizeof(TW),
                                 &fwd, &unpack_bank, &unpack_y, &corr, &export_bank, &export_y};
    return &ks;
  }
};

template <typename T, typename TW>
const KernelSet* pick_m(uint32_t m) {
  switch (m) {
    case 512: return Impl<T, TW, typename CfgFor<T, 512>::F>::get();
    case 1024: return Impl<T, TW, typename CfgFor<T, 1024>::F>::get();
    case 2048: return Impl<T, TW, typename CfgFor<T, 2048>::F>::get();
    case 4096: return Impl<T, TW, typename CfgFor<T, 4096>::F>::get();
    default: break;
  }
  if constexpr (std::is_same_v<T, float>) {
    switch (m) {
      case 8192: return Impl<T, TW, typename CfgFor<T, 8192>::F>::get();
      case 16384: return Impl<T, TW, typename CfgFor<T, 16384>::F>::get();
      case 32768: return Impl<T, TW, typename CfgFor<T, 32768>::F>::get();
      default: break;
    }
  }
  return nullptr;
}

const KernelSet* pick_kernels(bfs_precision p, uint32_t m) {
  switch (p) {
    case BFS_FP64: return pick_m<double, cx<double>>(m);
    case BFS_FP32: return pick_m<float, cx<float>>(m);
    case BFS_FP32_W16F: return pick_m<float, __half2>(m);
    case BFS_FP32_W16B: return pick_m<float, bf16x2>(m);
  }
  return nullptr;
}

// ----------------------------------------------------------------- tables --
// exp(+2 pi i num / den) rounded from long double.
void twiddle(uint64_t num, uint64_t den, long double& c, long double& s) {
  const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)(num % den) / (long double)den;
  c = cosl(ang);
  s = sinl(ang);
}

template <typename T>
std::vector<T> make_tables(const KernelSet& ks, uint32_t n) {
  // layout: tw_u [M] | tw1 [R1][S1] | tw2 [R2][R3], interleaved (re, im)
  const uint32_t M = ks.M, S1 = ks.R2 * ks.R3;
  std::vector<T> out(2ull * (M + uint64_t(ks.R1) * S1 + S1));
  size_t o = 0;
  long double c, s;
  for (uint32_t k = 0; k < M; ++k) {
    twiddle(k, n, c, s);
    out[o++] = T(c);
    out[o++] = T(s);
  }
  for (uint32_t n0 = 0; n0 < uint32_t(ks.R1); ++n0)
    for (uint32_t col = 0; col < S1; ++col) {
      twiddle(uint64_t(n0) * col, M, c, s);
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

struct JobBuffers {
  uint32_t S = 0;
  void* y = nullptr;          // [S][M] packed complex T
  double* sigma = nullptr;    // [S][K]
  tail_rec* tails = nullptr;  // [cap]
  unsigned long long* counter = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  uint64_t bytes = 0;
};

}  // namespace

struct bfs_plan {
  int device = 0;
  uint32_t N = 0, M = 0, K = 0;
  bfs_precision prec = BFS_FP32;
  double kappa = 0.0;
  uint64_t cap = 0;
  const KernelSet* ks = nullptr;
  void* bank = nullptr;
  void* tables = nullptr;
  const void* tw_u = nullptr;
  const void* tw1 = nullptr;
  const void* tw2 = nullptr;
  uint64_t bank_bytes = 0, plan_bytes = 0, budget = 0;
  hipStream_t copy_stream = nullptr;
  std::mutex mu;
  std::vector<JobBuffers*> pool;
  uint64_t live_job_bytes = 0;
  int live_jobs = 0;
};

struct bfs_job {
  bfs_plan* plan = nullptr;
  JobBuffers* buf = nullptr;
  hipStream_t stream = nullptr;
  uint32_t S = 0;
};

namespace {

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return BFS_ERR_HIP; \
  } while (0)

bfs_status alloc_checked(void** p, uint64_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return BFS_ERR_OUT_OF_MEMORY;
  }
  return BFS_OK;
}

void free_job_buffers(JobBuffers* b) {
  if (!b) return;
  if (b->y) (void)hipFree(b->y);
  if (b->sigma) (void)hipFree(b->sigma);
  if (b->tails) (void)hipFree(b->tails);
  if (b->counter) (void)hipFree(b->counter);
  for (auto& e : b->ev)
    if (e) (void)hipEventDestroy(e);
  delete b;
}

void free_plan(bfs_plan* p) {
  if (!p) return;
  for (auto* b : p->pool) free_job_buffers(b);
  p->pool.clear();
  if (p->bank) (void)hipFree(p->bank);
  if (p->tables) (void)hipFree(p->tables);
  if (p->copy_stream) (void)hipStreamDestroy(p->copy_stream);
  delete p;
}

bfs_status validate(const bfs_plan_desc* d) {
  if (!d) return BFS_ERR_INVALID_ARG;
  if (!is_pow2(d->n) || d->n < 2) return BFS_ERR_INVALID_ARG;
  if (!(d->fs > 0.0) || !std::isfinite(d->fs)) return BFS_ERR_INVALID_ARG;
  if (!(d->kappa >= 0.0) || !std::isfinite(d->kappa)) return BFS_ERR_INVALID_ARG;
  if (d->tail_capacity < 1) return BFS_ERR_INVALID_ARG;
  if (d->precision < BFS_FP64 || d->precision > BFS_FP32_W16B) return BFS_ERR_INVALID_ARG;
  if (d->taper > 1) return BFS_ERR_INVALID_ARG;
  if (d->explicit_templates) {
    if (d->n_explicit < 1 || d->explicit_len < 1 || d->explicit_len > d->n) return BFS_ERR_INVALID_ARG;
  } else {
    if (d->n_f0 < 1 || d->n_fdot < 1) return BFS_ERR_INVALID_ARG;
    if (uint64_t(d->n_f0) * d->n_fdot > 0xffffffffull) return BFS_ERR_INVALID_ARG;
    if (d->n_tau < 1 || !d->tau) return BFS_ERR_INVALID_ARG;
    for (double v : {d->f0_lo, d->f0_hi, d->fdot_lo, d->fdot_hi})
      if (!std::isfinite(v)) return BFS_ERR_INVALID_ARG;
    for (uint32_t i = 0; i < d->n_tau; ++i) {
      if (!(d->tau[i] > 0.0) || !std::isfinite(d->tau[i])) return BFS_ERR_INVALID_ARG;
      const double L = std::nearbyint(d->tau[i] * d->fs);
      if (L < 1.0 || L > double(d->n)) return BFS_ERR_INVALID_ARG;
    }
  }
  if (!pick_kernels(d->precision, d->n / 2)) return BFS_ERR_UNSUPPORTED;
  return BFS_OK;
}

bfs_status build_bank(bfs_plan* p, const bfs_plan_desc* d) {
  const KernelSet& ks = *p->ks;
  const uint32_t K = p->K, M = p->M;
  const bool expl = d->explicit_templates != nullptr;
  // per-template parameters (chirps) or the explicit bank, uploaded once
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
  // scratch for complex Z of a chunk of templates, plus per-template norms
  const uint64_t row_bytes = uint64_t(M) * 2 * ks.real_size;
  const uint64_t avail = p->budget > p->plan_bytes + param_bytes ? p->budget - p->plan_bytes - param_bytes : 0;
  uint64_t chunk = std::min<uint64_t>(K, std::max<uint64_t>(1, std::min<uint64_t>(4096, avail / (2 * row_bytes + 8))));
  if (avail < row_bytes + 8) return BFS_ERR_OUT_OF_MEMORY;
  void* scratch = nullptr;
  double* norms = nullptr;
  bfs_status st = alloc_checked(&params, param_bytes);
  if (st != BFS_OK) return st;
  st = alloc_checked(&scratch, chunk * row_bytes);
  if (st == BFS_OK) st = alloc_checked(reinterpret_cast<void**>(&norms), chunk * sizeof(double));
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
        a.tw1 = p->tw1;
        a.tw2 = p->tw2;
        a.out = scratch;
        a.inv_norm = norms;
        ok = ks.fwd(expl ? SRC_EXPLICIT : SRC_CHIRP, nb, s, a) == hipSuccess;
        ok = ok && ks.unpack_bank(nb, s, scratch, p->bank, expl ? nullptr : norms, p->tw_u, j0) == hipSuccess;
      }
      if (!ok) break;
      if (hipStreamSynchronize(s) != hipSuccess) break;
      out = BFS_OK;
    } while (false);
  }
  if (params) (void)hipFree(params);
  if (scratch) (void)hipFree(scratch);
  if (norms) (void)hipFree(norms);
  return out;
}

bfs_status get_job_buffers(bfs_plan* p, uint32_t S, JobBuffers** out) {
  std::lock_guard<std::mutex> lk(p->mu);
  for (size_t i = 0; i < p->pool.size(); ++i) {
    if (p->pool[i]->S >= S) {
      *out = p->pool[i];
      p->pool.erase(p->pool.begin() + long(i));
      p->live_job_bytes += (*out)->bytes;
      ++p->live_jobs;
      return BFS_OK;
    }
  }
  const uint64_t ybytes = uint64_t(S) * p->M * 2 * p->ks->real_size;
  const uint64_t sbytes = uint64_t(S) * p->K * sizeof(double);
  const uint64_t tbytes = p->cap * sizeof(tail_rec);
  const uint64_t need = ybytes + sbytes + tbytes + 256;
  // drop pooled buffers that are too small before asking for new memory
  for (auto* b : p->pool) free_job_buffers(b);
  p->pool.clear();
  if (p->plan_bytes + p->live_job_bytes + need > p->budget) return BFS_ERR_OUT_OF_MEMORY;
  auto* b = new (std::nothrow) JobBuffers();
  if (!b) return BFS_ERR_OUT_OF_MEMORY;
  b->S = S;
  b->bytes = need;
  bfs_status st = alloc_checked(&b->y, ybytes);
  if (st == BFS_OK) st = alloc_checked(reinterpret_cast<void**>(&b->sigma), sbytes);
  if (st == BFS_OK) st = alloc_checked(reinterpret_cast<void**>(&b->tails), tbytes);
  if (st == BFS_OK) st = alloc_checked(reinterpret_cast<void**>(&b->counter), 256);
  for (int i = 0; i < 4 && st == BFS_OK; ++i)
    if (hipEventCreate(&b->ev[i]) != hipSuccess) st = BFS_ERR_HIP;
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
}

// segment spectra: forward real FFT of each segment into the job's Y buffer
bfs_status queue_segment_fft(bfs_plan* p, const void* y_dev, uint32_t S, void* ybuf, hipStream_t st) {
  FwdArgs a{};
  a.src = y_dev;
  a.src_stride = p->N;
  a.src_len = p->N;
  a.tw1 = p->tw1;
  a.tw2 = p->tw2;
  a.out = ybuf;
  HIP_TRY(p->ks->fwd(SRC_SAMPLES, S, st, a));
  HIP_TRY(p->ks->unpack_y(S, st, ybuf, p->tw_u));
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
  p->N = d->n;
  p->M = d->n / 2;
  p->K = d->explicit_templates ? d->n_explicit : d->n_f0 * d->n_fdot;
  p->prec = d->precision;
  p->kappa = d->kappa;
  p->cap = d->tail_capacity;
  p->ks = pick_kernels(d->precision, p->M);
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
  p->budget = d->hbm_budget_bytes ? std::min<uint64_t>(d->hbm_budget_bytes, free_b) : free_b;
  if (hipStreamCreateWithFlags(&p->copy_stream, hipStreamNonBlocking) != hipSuccess) {
    delete p;
    return BFS_ERR_HIP;
  }
  const KernelSet& ks = *p->ks;
  p->bank_bytes = uint64_t(p->K) * p->M * ks.spec_size;
  const size_t n_tab = 2ull * (p->M + uint64_t(ks.R1) * ks.R2 * ks.R3 + uint64_t(ks.R2) * ks.R3);
  const uint64_t tab_bytes = n_tab * ks.real_size;
  p->plan_bytes = p->bank_bytes + tab_bytes;
  if (p->plan_bytes > p->budget) {
    free_plan(p);
    return BFS_ERR_OUT_OF_MEMORY;
  }
  bfs_status st = alloc_checked(&p->bank, p->bank_bytes);
  if (st == BFS_OK) st = alloc_checked(&p->tables, tab_bytes);
  if (st != BFS_OK) {
    free_plan(p);
    return st;
  }
  if (ks.real_size == sizeof(double)) {
    auto tab = make_tables<double>(ks, p->N);
    st = hipMemcpy(p->tables, tab.data(), tab_bytes, hipMemcpyHostToDevice) == hipSuccess ? BFS_OK : BFS_ERR_HIP;
  } else {
    auto tab = make_tables<float>(ks, p->N);
    st = hipMemcpy(p->tables, tab.data(), tab_bytes, hipMemcpyHostToDevice) == hipSuccess ? BFS_OK : BFS_ERR_HIP;
  }
  if (st != BFS_OK) {
    free_plan(p);
    return st;
  }
  const char* tb = static_cast<const char*>(p->tables);
  p->tw_u = tb;
  p->tw1 = tb + 2ull * p->M * ks.real_size;
  p->tw2 = tb + 2ull * (p->M + uint64_t(ks.R1) * ks.R2 * ks.R3) * ks.real_size;
  st = build_bank(p, d);
  if (st != BFS_OK) {
    free_plan(p);
    return st;
  }
  *out = p;
  return BFS_OK;
}

bfs_status bfsearch_plan_get_info(const bfs_plan* p, bfs_plan_info* out) {
  if (!p || !out) return BFS_ERR_INVALID_ARG;
  out->n = p->N;
  out->m = p->M;
  out->k = p->K;
  out->threads_per_correlation = uint32_t(p->ks->NT);
  out->bank_bytes = p->bank_bytes;
  out->plan_bytes = p->plan_bytes;
  out->precision = uint32_t(p->prec);
  out->reserved = 0;
  return BFS_OK;
}

bfs_status bfsearch_filter(bfs_plan* p, const void* y_dev, uint32_t S, void* hip_stream, bfs_job** out) {
  if (!out) return BFS_ERR_INVALID_ARG;
  *out = nullptr;
  if (!p || !y_dev || S < 1 || S > 65535) return BFS_ERR_INVALID_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return BFS_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  JobBuffers* b = nullptr;
  bfs_status rs = get_job_buffers(p, S, &b);
  if (rs != BFS_OK) return rs;
  auto fail = [&](bfs_status e) {
    put_job_buffers(p, b);
    return e;
  };
  if (hipEventRecord(b->ev[0], st) != hipSuccess) return fail(BFS_ERR_HIP);
  hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(64), 0, st, b->counter, uint64_t(1), 0ull);
  if (hipGetLastError() != hipSuccess) return fail(BFS_ERR_HIP);
  rs = queue_segment_fft(p, y_dev, S, b->y, st);
  if (rs != BFS_OK) return fail(rs);
  if (hipEventRecord(b->ev[1], st) != hipSuccess) return fail(BFS_ERR_HIP);
  CorrArgs a{};
  a.bank = p->bank;
  a.y = b->y;
  a.tw_u = p->tw_u;
  a.tw1 = p->tw1;
  a.tw2 = p->tw2;
  a.K = p->K;
  a.kappa = p->kappa;
  a.sigma = b->sigma;
  a.tails = b->tails;
  a.counter = b->counter;
  a.cap = p->cap;
  if (p->ks->corr(false, S, st, a) != hipSuccess) return fail(BFS_ERR_HIP);
  if (hipEventRecord(b->ev[2], st) != hipSuccess) return fail(BFS_ERR_HIP);
  if (hipEventRecord(b->ev[3], st) != hipSuccess) return fail(BFS_ERR_HIP);
  auto* j = new (std::nothrow) bfs_job();
  if (!j) return fail(BFS_ERR_OUT_OF_MEMORY);
  j->plan = p;
  j->buf = b;
  j->stream = st;
  j->S = S;
  *out = j;
  return BFS_OK;
}

bfs_status bfsearch_fetch_tails(bfs_job* j, bfs_tail* out_host, uint64_t capacity, uint64_t* n_written,
                                uint64_t* n_total) {
  if (!j || !n_written || !n_total || (capacity > 0 && !out_host)) return BFS_ERR_INVALID_ARG;
  bfs_plan* p = j->plan;
  if (hipSetDevice(p->device) != hipSuccess) return BFS_ERR_HIP;
  HIP_TRY(hipStreamWaitEvent(p->copy_stream, j->buf->ev[3], 0));
  unsigned long long count = 0;
  HIP_TRY(hipMemcpyAsync(&count, j->buf->counter, sizeof(count), hipMemcpyDeviceToHost, p->copy_stream));
  HIP_TRY(hipStreamSynchronize(p->copy_stream));
  const uint64_t on_dev = std::min<uint64_t>(count, p->cap);
  std::vector<bfs_tail> tmp(on_dev);
  if (on_dev) {
    HIP_TRY(hipMemcpyAsync(tmp.data(), j->buf->tails, on_dev * sizeof(bfs_tail), hipMemcpyDeviceToHost,
                           p->copy_stream));
    HIP_TRY(hipStreamSynchronize(p->copy_stream));
  }
  std::sort(tmp.begin(), tmp.end(), [](const bfs_tail& a, const bfs_tail& b) {
    if (a.segment != b.segment) return a.segment < b.segment;
    if (a.template_id != b.template_id) return a.template_id < b.template_id;
    return a.lag < b.lag;
  });
  const uint64_t nw = std::min<uint64_t>(on_dev, capacity);
  if (nw) std::memcpy(out_host, tmp.data(), nw * sizeof(bfs_tail));
  *n_written = nw;
  *n_total = count;
  return (count > nw) ? BFS_ERR_TAIL_OVERFLOW : BFS_OK;
}

bfs_status bfsearch_fetch_sigma(bfs_job* j, double* out_host) {
  if (!j || !out_host) return BFS_ERR_INVALID_ARG;
  bfs_plan* p = j->plan;
  if (hipSetDevice(p->device) != hipSuccess) return BFS_ERR_HIP;
  HIP_TRY(hipStreamWaitEvent(p->copy_stream, j->buf->ev[3], 0));
  HIP_TRY(hipMemcpyAsync(out_host, j->buf->sigma, uint64_t(j->S) * p->K * sizeof(double), hipMemcpyDeviceToHost,
                         p->copy_stream));
  HIP_TRY(hipStreamSynchronize(p->copy_stream));
  return BFS_OK;
}

bfs_status bfsearch_job_timing(bfs_job* j, float* corr_ms, float* total_ms) {
  if (!j || !corr_ms || !total_ms) return BFS_ERR_INVALID_ARG;
  HIP_TRY(hipEventSynchronize(j->buf->ev[3]));
  HIP_TRY(hipEventElapsedTime(corr_ms, j->buf->ev[1], j->buf->ev[2]));
  HIP_TRY(hipEventElapsedTime(total_ms, j->buf->ev[0], j->buf->ev[3]));
  return BFS_OK;
}

bfs_status bfsearch_job_release(bfs_job* j) {
  if (!j) return BFS_ERR_INVALID_ARG;
  // buffers may be reused by the next filter call: wait for this job's kernels
  (void)hipEventSynchronize(j->buf->ev[3]);
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

bfs_status bfsearch_correlate_dense(bfs_plan* p, const void* y_dev, uint32_t S, void* rho_dev, double* sigma_dev,
                                    void* hip_stream) {
  if (!p || !y_dev || !rho_dev || S < 1 || S > 65535) return BFS_ERR_INVALID_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return BFS_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  JobBuffers* b = nullptr;
  bfs_status rs = get_job_buffers(p, S, &b);
  if (rs != BFS_OK) return rs;
  rs = queue_segment_fft(p, y_dev, S, b->y, st);
  CorrArgs a{};
  a.bank = p->bank;
  a.y = b->y;
  a.tw_u = p->tw_u;
  a.tw1 = p->tw1;
  a.tw2 = p->tw2;
  a.K = p->K;
  a.kappa = p->kappa;
  a.sigma = sigma_dev;
  a.cap = 0;
  a.rho = rho_dev;
  if (rs == BFS_OK && p->ks->corr(true, S, st, a) != hipSuccess) rs = BFS_ERR_HIP;
  if (rs == BFS_OK && hipEventRecord(b->ev[3], st) != hipSuccess) rs = BFS_ERR_HIP;
  // the buffers go back to the pool only after the queued kernels finish
  if (rs == BFS_OK) (void)hipEventSynchronize(b->ev[3]);
  put_job_buffers(p, b);
  return rs;
}

bfs_status bfsearch_plan_spectra(const bfs_plan* p, uint32_t first, uint32_t count, double* out_dev,
                                 void* hip_stream) {
  if (!p || !out_dev || count < 1 || uint64_t(first) + count > p->K || count > 65535) return BFS_ERR_INVALID_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return BFS_ERR_HIP;
  HIP_TRY(p->ks->export_bank(count, static_cast<hipStream_t>(hip_stream), p->bank, out_dev, first));
  return BFS_OK;
}

bfs_status bfsearch_job_spectra(const bfs_job* j, double* out_dev) {
  if (!j || !out_dev) return BFS_ERR_INVALID_ARG;
  if (hipSetDevice(j->plan->device) != hipSuccess) return BFS_ERR_HIP;
  HIP_TRY(j->plan->ks->export_y(j->S, j->stream, j->buf->y, out_dev));
  return BFS_OK;
}

}  // extern "C"
