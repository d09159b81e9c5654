// Kernel sets of the matched-filter library: one per (real type, spectrum
// storage type, transform shape, split, load-group depth).  A set bundles the
// host launchers of its forward transform, unpack, fused correlation (single
// segments and detector pairs) and export kernels behind function pointers,
// so the runtime picks a set per segment length at plan time.  Each storage
// precision's sets are instantiated in a source of their own (bfs_ks_*.hip),
// which keeps the build parallel.
#pragma once

#include <hip/hip_ext.h>

#include <algorithm>
#include <type_traits>

#include "bfs_fused.h"

// A correlation launch that carries the job's timing events in its own dispatch
// (E0 recorded as the kernel starts, E1 as it ends) when either is given, instead
// of as separate packets between the kernels on the stream.
#define BFS_LAUNCH_TIMED(K, GRID, BLOCK, ST, E0, E1, ...)                      \
  do {                                                                       \
    if ((E0) || (E1))                                                        \
      hipExtLaunchKernelGGL(K, GRID, BLOCK, 0, ST, E0, E1, 0, __VA_ARGS__);   \
    else                                                                     \
      hipLaunchKernelGGL(K, GRID, BLOCK, 0, ST, __VA_ARGS__);                \
  } while (0)

namespace bfs {

// ---------------------------------------------------------------- kernels --
// A kernel configuration per (real type, storage type, M = N/2): radices
// R1*R2*R3 and threads per workgroup of the on-chip transform, whether the
// length-M inverse transform runs as two halves (split, when M points do not
// fit one workgroup's registers), and the load-group depth G of the product
// stage.  Each M has a short list of candidates; the first is the default and
// the autotuner may pick another by timing (see tune_size).
struct FwdArgs {
  const void* src;          // explicit templates [K][src_stride] (FP64); segments packed
                            // back to back at src_stride samples when seg_ptr is null
  uint64_t src_stride;
  uint32_t src_len;
  const uint64_t* seg_ptr;  // segment sources: device address of each item's samples
  const double* f0;
  const double* fdot;
  const uint32_t* len;
  double fs;
  int taper;
  uint32_t first;
  const void* tw1;
  const void* tw2;
  void* out;
  double* energy;
  uint32_t zs;  // > 1: segments' transforms split zs ways (sub-sequence b mod zs of segment b / zs)
  unsigned long long* zero;  // not null: three counters the launch's first workgroup clears
};

struct CorrArgs {
  const void* bank;
  const void* y;
  const uint32_t* seg_ids;  // global segment id of each grid row (null: the row index)
  const void* tw_u;
  const void* tw1;
  const void* tw2;
  uint32_t K;
  uint32_t tile;            // segments per tile of the workgroup order (1 <= tile <= rows)
  double kappa;
  double* sigma;
  void* tails;              // tail records of the set's type (tail_rec_t of its real type)
  unsigned long long* counter;
  uint64_t cap;
  unsigned long long* proj;  // projection keys (null: tail list)
  const uint64_t* proj_off;  // per grid row: offset of its lags in proj
  double kappa_hi;           // > 0: upper edge of a finite tail band
  void* rho;
  // fused synthesis (corr_fused): grid parameters and unit-norm factors of every template,
  // the sample rate, taper and symmetry, and the input rows of the pruned first pass
  const double* f0;
  const double* fdot;
  const uint32_t* len;
  const float* norm;
  double fs;
  int taper;
  int sym;
  uint32_t rows;
  uint32_t cus;  // compute units of the device (looping sets size their grid by it; 0: one item per workgroup)
  // timing events of the job (may be null): ev_start with the call's first launch, ev_stop
  // with each launch, so the last one's end stands
  hipEvent_t ev_start = nullptr;
  hipEvent_t ev_stop = nullptr;
};

struct KernelSet {
  int R1, R2, R3, NT;
  int FM;            // length of the on-chip transform
  int M;             // N/2 (= FM, or 2 FM when split)
  int split;
  int G;             // load-group depth of the product stage
  int loop;          // 1: workgroups loop over correlations (corr_loop_kernel)
  size_t real_size;  // sizeof(T)
  size_t spec_size;  // bytes of one stored template spectrum element
  size_t tail_size;  // bytes of one tail record the kernels write
  hipError_t (*fwd)(int src, uint32_t batch, hipStream_t st, const FwdArgs& a);
  hipError_t (*unpack_bank)(uint32_t batch, hipStream_t st, const void* Z, void* out, const double* energy,
                            const void* tw_u, uint64_t row_off);
  hipError_t (*unpack_y)(uint32_t batch, hipStream_t st, const void* Z, void* out, const void* tw_u);
  hipError_t (*corr)(bool dense, uint32_t S, hipStream_t st, const CorrArgs& a);
  // detector pairs (S = 2 x pairs rows, pair q at rows 2q, 2q + 1); null for split sets
  hipError_t (*corr_pair)(bool dense, uint32_t S, hipStream_t st, const CorrArgs& a);
  hipError_t (*export_bank)(uint32_t count, hipStream_t st, const void* bank, double* out, uint64_t first);
  hipError_t (*export_y)(uint32_t count, hipStream_t st, const void* y, double* out);
  // fused synthesis (FP32 cubic sets with load group 4; null otherwise): the correlation with
  // each template made on chip, and the segment spectra's copy in the fused layout
  // the join of segment transforms split JOIN_A ways (JOIN_A = M / 1024 > 1, unsplit sets; 0: none)
  hipError_t (*join)(uint32_t count, hipStream_t st, const void* in, void* out, const void* tw_u);
  int join_a;
  hipError_t (*corr_fused)(bool dense, uint32_t S, hipStream_t st, const CorrArgs& a);
  hipError_t (*permute_y)(uint32_t count, hipStream_t st, const void* y, void* out);
  int fused_rows_max;  // largest pruned first-pass row count built below the full R1
};

template <typename T, typename TW, class F, int SPLIT, int G, int LOOP = 0>
struct Impl {
  static_assert(!LOOP || !SPLIT, "looping workgroups are built for unsplit transforms");
  static constexpr int M = F::M * (SPLIT ? 2 : 1);
  static hipError_t fwd(int src, uint32_t batch, hipStream_t st, const FwdArgs& a) {
    const dim3 grid(batch * (SPLIT ? 2u : 1u)), block(F::NT);
    const auto* t1 = static_cast<const cx<T>*>(a.tw1);
    const auto* t2 = static_cast<const cx<T>*>(a.tw2);
    auto* out = static_cast<cx<T>*>(a.out);
    if (src == SRC_SAMPLES)
      hipLaunchKernelGGL((fwd_fft_kernel<T, F, SRC_SAMPLES>), grid, block, 0, st, a.src, a.src_stride, a.src_len,
                         a.seg_ptr, a.f0, a.fdot, a.len, a.fs, a.taper, a.first, t1, t2, out, a.energy, SPLIT, a.zs, a.zero);
    else if (src == SRC_CHIRP)
      hipLaunchKernelGGL((fwd_fft_kernel<T, F, SRC_CHIRP>), grid, block, 0, st, a.src, a.src_stride, a.src_len,
                         a.seg_ptr, a.f0, a.fdot, a.len, a.fs, a.taper, a.first, t1, t2, out, a.energy, SPLIT, a.zs, a.zero);
    else if (src == SRC_CHIRP_SYM)
      hipLaunchKernelGGL((fwd_fft_kernel<T, F, SRC_CHIRP_SYM>), grid, block, 0, st, a.src, a.src_stride, a.src_len,
                         a.seg_ptr, a.f0, a.fdot, a.len, a.fs, a.taper, a.first, t1, t2, out, a.energy, SPLIT, a.zs, a.zero);
    else
      hipLaunchKernelGGL((fwd_fft_kernel<T, F, SRC_EXPLICIT>), grid, block, 0, st, a.src, a.src_stride, a.src_len,
                         a.seg_ptr, a.f0, a.fdot, a.len, a.fs, a.taper, a.first, t1, t2, out, a.energy, SPLIT, a.zs, a.zero);
    return hipGetLastError();
  }
  static hipError_t unpack_bank(uint32_t batch, hipStream_t st, const void* Z, void* out, const double* energy,
                                const void* tw_u, uint64_t row_off) {
    const dim3 grid((M / 2 + 1 + 255) / 256, batch);
    hipLaunchKernelGGL((rfft_unpack_kernel<T, TW>), grid, dim3(256), 0, st, static_cast<const cx<T>*>(Z),
                       static_cast<TW*>(out), energy, static_cast<const cx<T>*>(tw_u), uint32_t(M), row_off, SPLIT);
    return hipGetLastError();
  }
  static hipError_t unpack_y(uint32_t batch, hipStream_t st, const void* Z, void* out, const void* tw_u) {
    const dim3 grid((M / 2 + 1 + 255) / 256, batch);
    hipLaunchKernelGGL((rfft_unpack_kernel<T, cx<T>>), grid, dim3(256), 0, st, static_cast<const cx<T>*>(Z),
                       static_cast<cx<T>*>(out), static_cast<const double*>(nullptr),
                       static_cast<const cx<T>*>(tw_u), uint32_t(M), uint64_t(0), SPLIT);
    return hipGetLastError();
  }
  // fused synthesis is built for FP32 cubic transforms with one column per thread, load group 4
  static constexpr bool FUSED = !SPLIT && std::is_same_v<T, float> && std::is_same_v<TW, cx<T>> && G == 4 &&
                                fused_shape<F>();
  static constexpr int FUSED_NZ = F::R1 > 2 ? 2 : F::R1;  // the pruned first pass (rows < 2 S1)
  enum Mode { MODE_SINGLE = 0, MODE_PAIR = 1, MODE_FUSED = 2 };
  template <bool DENSE, int NZ>
  static void launch_fused(uint32_t blocks, const cx<T>* y, const uint32_t* seg_ids, const uint64_t* proj_off,
                           uint32_t kn, uint32_t rn, uint32_t tile, uint32_t j0, uint32_t row0, hipStream_t st,
                           const CorrArgs& a, hipEvent_t e0, hipEvent_t e1) {
    if constexpr (FUSED) {
      BFS_LAUNCH_TIMED((corr_fused_kernel<T, F, DENSE, G, NZ>), dim3(blocks), dim3(F::NT), st, e0, e1, y, seg_ids,
                         static_cast<const cx<T>*>(a.tw_u), static_cast<const cx<T>*>(a.tw1),
                         static_cast<const cx<T>*>(a.tw2), a.f0 + j0, a.fdot + j0, a.len + j0, a.norm + j0, a.fs,
                         a.taper, a.sym, kn, rn, tile, a.kappa, a.sigma, static_cast<tail_rec_t<T>*>(a.tails),
                         a.counter, a.cap, a.proj, proj_off, a.kappa_hi, DENSE ? static_cast<T*>(a.rho) : nullptr, j0,
                         a.K, row0);
    }
  }
  template <bool DENSE, int MODE>
  static void launch_corr(uint32_t blocks, const TW* bank, const cx<T>* y, const uint32_t* seg_ids,
                          const uint64_t* proj_off, uint32_t kn, uint32_t rn, uint32_t tile, uint32_t j0,
                          uint32_t row0, hipStream_t st, const CorrArgs& a, hipEvent_t e0, hipEvent_t e1) {
    const auto* tu = static_cast<const cx<T>*>(a.tw_u);
    const auto* t1 = static_cast<const cx<T>*>(a.tw1);
    const auto* t2 = static_cast<const cx<T>*>(a.tw2);
    T* rho = DENSE ? static_cast<T*>(a.rho) : nullptr;
    auto* tails = static_cast<tail_rec_t<T>*>(a.tails);
    constexpr bool PAIR = MODE == MODE_PAIR;
    if constexpr (MODE == MODE_FUSED) {
      if (a.rows <= uint32_t(FUSED_NZ))
        launch_fused<DENSE, FUSED_NZ>(blocks, y, seg_ids, proj_off, kn, rn, tile, j0, row0, st, a, e0, e1);
      else
        launch_fused<DENSE, F::R1>(blocks, y, seg_ids, proj_off, kn, rn, tile, j0, row0, st, a, e0, e1);
    } else if constexpr (LOOP && !PAIR && !SPLIT) {
      BFS_LAUNCH_TIMED((corr_loop_kernel<T, TW, F, DENSE, G>), dim3(loop_grid(blocks, a.cus)), dim3(F::NT), st, e0,
                       e1, bank, y, seg_ids, tu, t1, t2, kn, rn, tile, a.kappa, a.sigma, tails, a.counter, a.cap,
                         a.proj, proj_off, a.kappa_hi, rho, j0, a.K, row0, blocks);
    } else if constexpr (PAIR && !SPLIT)
      BFS_LAUNCH_TIMED((pair_kernel<T, TW, F, DENSE, G>), dim3(blocks), dim3(F::NT), st, e0, e1, bank, y, seg_ids, tu,
                         t1, t2, kn, rn, tile, a.kappa, a.sigma, tails, a.counter, a.cap, a.proj, proj_off,
                         a.kappa_hi, rho, j0, a.K, row0);
    else if constexpr (SPLIT)
      BFS_LAUNCH_TIMED((corr2_kernel<T, TW, F, DENSE, G>), dim3(blocks), dim3(F::NT), st, e0, e1, bank, y, seg_ids, tu,
                         t1, t2, kn, rn, tile, a.kappa, a.sigma, tails, a.counter, a.cap, a.proj, proj_off,
                         a.kappa_hi, rho, j0, a.K, row0);
    else
      BFS_LAUNCH_TIMED((corr_kernel<T, TW, F, DENSE, G>), dim3(blocks), dim3(F::NT), st, e0, e1, bank, y, seg_ids, tu,
                         t1, t2, kn, rn, tile, a.kappa, a.sigma, tails, a.counter, a.cap, a.proj, proj_off,
                         a.kappa_hi, rho, j0, a.K, row0);
  }
  // Looping sets: as many workgroups as the device holds at once (a multiple of 8, so
  // each keeps the XCD of its items), at most one per item.
  static uint32_t loop_grid(uint32_t items, uint32_t cus) {
    static int per_cu = -1;
    if (per_cu < 0) {
      int occ = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, corr_loop_kernel<T, TW, F, false, G>, F::NT, 0) !=
          hipSuccess) {
        (void)hipGetLastError();
        occ = 1;
      }
      per_cu = std::max(occ, 1);
    }
    if (!cus) return items;
    const uint32_t g = std::max<uint32_t>(8, (cus * uint32_t(per_cu)) & ~7u);
    return std::min(items, g);
  }
  // 1-D grids in the XCD-aware order of tile_map, 8 ceil(K/8) S workgroups in all.  A
  // launch holds at most MAX_ITEMS work items (the dispatch's grid size is a 32-bit count
  // of work items): larger jobs run as several launches over slices of the segment rows
  // (each with every template), and of the bank too when one row alone is too large.
  static constexpr uint64_t MAX_ITEMS = 1ull << 31;
  template <int MODE>
  static hipError_t corr_t(bool dense, uint32_t S, hipStream_t st, const CorrArgs& a) {
    constexpr bool PAIR = MODE == MODE_PAIR;
    if (!S || !a.K || (PAIR && (S & 1u))) return hipErrorInvalidValue;
    const uint64_t max_blocks = MAX_ITEMS / F::NT;
    uint64_t kc = a.K;  // templates per launch: all, or a multiple of 8 that fits one row
    if (8ull * ((kc + 7) / 8) > max_blocks) kc = (max_blocks / 8) * 8;
    const auto* bank = static_cast<const TW*>(a.bank);
    const auto* y = static_cast<const cx<T>*>(a.y);
    hipEvent_t e0 = a.ev_start;  // with the first launch only
    for (uint64_t j0 = 0; j0 < a.K; j0 += kc) {
      const uint32_t kn = uint32_t(std::min<uint64_t>(kc, a.K - j0));
      const uint64_t per_row = 8ull * ((kn + 7) / 8);
      uint32_t rows = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(S, max_blocks / per_row)));
      if (PAIR) rows = std::max<uint32_t>(2, rows & ~1u);  // a pair's two rows stay in one launch
      for (uint32_t r0 = 0; r0 < S; r0 += rows) {
        const uint32_t rn = std::min(rows, S - r0);
        const uint32_t tile = std::min<uint32_t>(std::max<uint32_t>(a.tile, 1u), rn);
        const uint32_t blocks = uint32_t(per_row * rn);
        const TW* bk = bank ? bank + j0 * uint64_t(M) : nullptr;
        const cx<T>* yr = y + uint64_t(r0) * M;
        const uint32_t* ids = a.seg_ids ? a.seg_ids + r0 : nullptr;
        const uint64_t* po = a.proj_off ? a.proj_off + r0 : nullptr;
        if (dense)
          launch_corr<true, MODE>(blocks, bk, yr, ids, po, kn, rn, tile, uint32_t(j0), r0, st, a, e0, a.ev_stop);
        else
          launch_corr<false, MODE>(blocks, bk, yr, ids, po, kn, rn, tile, uint32_t(j0), r0, st, a, e0, a.ev_stop);
        e0 = nullptr;
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
    }
    return hipSuccess;
  }
  static hipError_t corr(bool dense, uint32_t S, hipStream_t st, const CorrArgs& a) {
    return corr_t<MODE_SINGLE>(dense, S, st, a);
  }
  static hipError_t corr_pair(bool dense, uint32_t S, hipStream_t st, const CorrArgs& a) {
    return corr_t<MODE_PAIR>(dense, S, st, a);
  }
  static hipError_t corr_fused(bool dense, uint32_t S, hipStream_t st, const CorrArgs& a) {
    if (!a.f0 || !a.fdot || !a.len || !a.norm || a.rows < 1 || a.rows > uint32_t(F::R1)) return hipErrorInvalidValue;
    return corr_t<MODE_FUSED>(dense, S, st, a);
  }
  static constexpr int JOIN_A = (!SPLIT && M >= 2048 && M <= 32768) ? M / 1024 : 0;
  static hipError_t join(uint32_t count, hipStream_t st, const void* in, void* out, const void* tw_u) {
    if constexpr (JOIN_A > 1) {
      const dim3 grid(uint32_t(M) / 256, count);
      hipLaunchKernelGGL((fft_join_kernel<T, JOIN_A>), grid, dim3(256), 0, st, static_cast<const cx<T>*>(in),
                         static_cast<cx<T>*>(out), static_cast<const cx<T>*>(tw_u), uint32_t(M));
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  static hipError_t permute_y(uint32_t count, hipStream_t st, const void* y, void* out) {
    if constexpr (FUSED) {
      const dim3 grid((M + 255) / 256, count);
      hipLaunchKernelGGL((fused_permute_kernel<T, F::R1>), grid, dim3(256), 0, st, static_cast<const cx<T>*>(y),
                         static_cast<cx<T>*>(out));
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  static hipError_t export_bank(uint32_t count, hipStream_t st, const void* bank, double* out, uint64_t first) {
    const dim3 grid((M + 1 + 255) / 256, count);
    hipLaunchKernelGGL((spectrum_export_kernel<T, TW>), grid, dim3(256), 0, st, static_cast<const TW*>(bank), out,
                       uint32_t(M), first, SPLIT);
    return hipGetLastError();
  }
  static hipError_t export_y(uint32_t count, hipStream_t st, const void* y, double* out) {
    const dim3 grid((M + 1 + 255) / 256, count);
    hipLaunchKernelGGL((spectrum_export_kernel<T, cx<T>>), grid, dim3(256), 0, st, static_cast<const cx<T>*>(y),
                       out, uint32_t(M), uint64_t(0), SPLIT);
    return hipGetLastError();
  }
  static const KernelSet* get() {
    static const KernelSet ks = {F::R1, F::R2, F::R3, F::NT, F::M, M, SPLIT, G, LOOP, sizeof(T), sizeof(TW),
                                 sizeof(tail_rec_t<T>), &fwd, &unpack_bank, &unpack_y, &corr, SPLIT ? nullptr : &corr_pair, &export_bank,
                                 &export_y, JOIN_A > 1 ? &join : nullptr, JOIN_A, FUSED ? &corr_fused : nullptr,
                                 FUSED ? &permute_y : nullptr, FUSED_NZ};
    return &ks;
  }
};

constexpr int MAX_CANDIDATES = 8;

struct Candidates {
  const KernelSet* ks[MAX_CANDIDATES];
  int count = 0;
  template <typename T, typename TW, class F, int SPLIT, int G, int LOOP = 0>
  void add() {
    if (count < MAX_CANDIDATES) ks[count++] = Impl<T, TW, F, SPLIT, G, LOOP>::get();
  }
};

template <typename T, typename TW>
Candidates candidates_t(uint32_t m) {
  constexpr bool F32 = std::is_same_v<T, float>;
  Candidates c;
  switch (m) {
    case 512:
      c.add<T, TW, Fft3<T, 8, 8, 8, 64>, 0, 4>();
      c.add<T, TW, Fft3<T, 8, 8, 8, 64>, 0, 2>();
      break;
    case 1024:
      c.add<T, TW, Fft3<T, 4, 16, 16, 64>, 0, 4>();
      c.add<T, TW, Fft3<T, 4, 16, 16, 64>, 0, 2>();
      break;
    case 2048:
      c.add<T, TW, Fft3<T, 8, 16, 16, 128>, 0, 4>();
      c.add<T, TW, Fft3<T, 8, 16, 16, 128>, 0, 2>();
      break;
    case 4096:
      c.add<T, TW, Fft3<T, 16, 16, 16, 256>, 0, 4>();
      c.add<T, TW, Fft3<T, 16, 16, 16, 256>, 0, 2>();
      if constexpr (F32) {
        c.add<T, TW, Fft3<T, 16, 16, 16, 128>, 0, 4>();
        c.add<T, TW, Fft3<T, 4, 32, 32, 128>, 0, 4>();
      }
      break;
    case 8192:
      if constexpr (F32) {
        c.add<T, TW, Fft3<T, 8, 32, 32, 256>, 0, 4>();
        c.add<T, TW, Fft3<T, 8, 32, 32, 256>, 0, 2>();
        c.add<T, TW, Fft3<T, 32, 16, 16, 256>, 0, 4>();
      } else {
        c.add<T, TW, Fft3<T, 16, 16, 16, 256>, 1, 4>();
        c.add<T, TW, Fft3<T, 16, 16, 16, 256>, 1, 2>();
      }
      break;
    case 16384:
      if constexpr (F32) {
        c.add<T, TW, Fft3<T, 16, 32, 32, 512>, 0, 4>();
        c.add<T, TW, Fft3<T, 16, 32, 32, 512>, 0, 2>();
      }
      break;
    case 32768:
      if constexpr (F32) {
        c.add<T, TW, Fft3<T, 32, 32, 32, 1024>, 0, 8>();
        c.add<T, TW, Fft3<T, 32, 32, 32, 1024>, 0, 4>();
        c.add<T, TW, Fft3<T, 32, 32, 32, 1024>, 0, 2>();
        c.add<T, TW, Fft3<T, 32, 32, 32, 1024>, 0, 8, 1>();
        c.add<T, TW, Fft3<T, 32, 32, 32, 1024>, 0, 4, 1>();
      }
      break;
    case 65536:
      if constexpr (F32) {
        c.add<T, TW, Fft3<T, 32, 32, 32, 1024>, 1, 4>();
        c.add<T, TW, Fft3<T, 32, 32, 32, 1024>, 1, 2>();
        c.add<T, TW, Fft3<T, 32, 32, 32, 1024>, 1, 8>();
      }
      break;
    default:
      break;
  }
  return c;
}

// The candidate sets of each storage precision (one source each).
Candidates candidates_f64(uint32_t m);
Candidates candidates_f32(uint32_t m);
Candidates candidates_w16f(uint32_t m);
Candidates candidates_w16b(uint32_t m);

}  // namespace bfs
