// Fused synthesis: the correlation kernel that makes each template's spectrum
// itself instead of reading it from a resident bank (for banks larger than
// the HBM budget, e.g. 2^20 FP32 spectra of 2^16-point transforms = 256 GiB).
//
// One workgroup per (template j, segment row), as corr_kernel:
//   1. synthesise w_j (FP64 phase reduced mod one cycle and FP64 taper, the
//      same chirp_sample as the resident bank's build; FP32 values) into the
//      forward transform's first pass; only the first NZ of its R rows can be
//      nonzero (the template is L <= N samples of the zero-padded N), so the
//      first radix-R pass is pruned to NZ inputs;
//   2. forward complex FFT of z_n = w_{2n} + i w_{2n+1} (length M = N/2) on
//      chip, with the pass-2/3 work assigned so that the result lands in the
//      layout the inverse transform starts from (below);
//   3. unpack Z -> W (the real spectrum, Hermitian partners by lane swaps),
//      scaled by the template's FP64-computed unit-norm factor;
//   4. C = conj(W) Y with the segment spectrum Y (L2-resident, stored in the
//      same layout), the FP64 Parseval sum, the Hermitian repack;
//   5. the inverse transform, threshold and compaction of corr_kernel.
// Nothing of the template touches HBM.
//
// Layout.  Cubic transforms only: R1 = R2 = R3 = R, NT = R^2 threads, one
// pass-1 column and one pass-2/3 item per thread.  The forward transform's
// output index is n = n0 + R m0 + R^2 m' with m' in registers; the inverse's
// pass-1 input index is k = col + S1 k2 with k2 in registers (S1 = R^2).  So a
// thread whose forward pass-3 item is (n0, m0) holds, after the forward
// transform, exactly inverse column col = n0 + R m0 with its R registers in
// order.  The inverse's Hermitian repack (and the unpack) needs column col
// and its partner S1 - col in lanes l and l ^ 32 of one wave, with register
// k2 partnered by R - 1 - k2 (column 0 and column S1/2 pair within their own
// thread), and the forward's wave-local pass-2 -> pass-3 exchange needs every
// n0 group inside one wave.  FusedMap assigns the items so both hold:
//   col = n0 + R m0 has partner (R - n0, R - 1 - m0) for n0 != 0, R/2;
//   (R/2, R - 1 - m0) for n0 = R/2; (0, R - m0) for n0 = 0 (m0 = 0 and
//   m0 = R/2 are their own partners, columns 0 and S1/2).
// The lower 32 lanes of each wave take representatives in the order
//   (0, 0..R/2-1), (R/2, 0..R/2-1), (1, 0..R-1), (2, 0..R-1), ..., (R/2-1, ..)
// and lane l + 32 takes the partner of lane l (lane 32 of wave 0: (0, R/2)).
// Lane 0 of wave 0 is column 0 and lane 32 is column S1/2, as in MAP_MIRROR,
// so the repack's fixups apply unchanged.  The segment spectrum is stored
// permuted so that a thread's R values are coalesced across the wave:
// element (thread t, register k2) at position k2 NT + t.
#pragma once

#include "bfs_kernels.h"

namespace bfs {

template <int R>
struct FusedMap {
  static constexpr int NT = R * R, S1 = R * R;
  static_assert(R >= 8 && (R & (R - 1)) == 0 && NT % 64 == 0, "cubic transform of whole waves");

  // representative (lower-lane) item of slot p < NT / 2
  static constexpr void slot_item(int p, int& n0, int& m0) {
    if (p < R / 2) {
      n0 = 0;
      m0 = p;
    } else if (p < R) {
      n0 = R / 2;
      m0 = p - R / 2;
    } else {
      n0 = 1 + (p - R) / R;
      m0 = (p - R) % R;
    }
  }
  // the item the upper lane of that slot holds
  static constexpr void partner(int n0, int m0, int& n1, int& m1) {
    if (n0 == 0) {
      n1 = 0;
      m1 = m0 == 0 ? R / 2 : R - m0;
    } else if (n0 == R / 2) {
      n1 = R / 2;
      m1 = R - 1 - m0;
    } else {
      n1 = R - n0;
      m1 = R - 1 - m0;
    }
  }
  static constexpr void item(int t, int& n0, int& m0) {
    const int l = t & 63;
    slot_item(32 * (t >> 6) + (l & 31), n0, m0);
    if (l >= 32) {
      const int a = n0, b = m0;
      partner(a, b, n0, m0);
    }
  }
  static constexpr int col(int t) {
    int n0 = 0, m0 = 0;
    item(t, n0, m0);
    return n0 + R * m0;
  }
  // the thread whose item is column c
  static constexpr int thread_of(int c) {
    const int n0 = c % R, m0 = c / R;
    int slot = 0;
    bool upper = false;
    if (n0 == 0) {
      if (m0 < R / 2) {
        slot = m0;
      } else if (m0 == R / 2) {
        slot = 0;
        upper = true;
      } else {
        slot = R - m0;
        upper = true;
      }
    } else if (n0 == R / 2) {
      if (m0 < R / 2) {
        slot = R / 2 + m0;
      } else {
        slot = R / 2 + (R - 1 - m0);
        upper = true;
      }
    } else if (n0 < R / 2) {
      slot = R + (n0 - 1) * R + m0;
    } else {
      slot = R + (R - n0 - 1) * R + (R - 1 - m0);
      upper = true;
    }
    return 64 * (slot / 32) + slot % 32 + (upper ? 32 : 0);
  }
  // Compile-time proof of the properties the kernel relies on: the map is a
  // bijection of threads onto columns, lanes l and l ^ 32 hold Hermitian
  // partners (except columns 0 and S1/2 in lanes 0 and 32 of wave 0), and
  // every n0 group lies in one wave.
  static constexpr bool valid() {
    for (int t = 0; t < NT; ++t) {
      const int c = col(t);
      if (c < 0 || c >= S1 || thread_of(c) != t) return false;
      if ((t & 63) < 32) {
        const int cp = col(t ^ 32);
        if (t == 0) {
          if (c != 0 || cp != S1 / 2) return false;
        } else if ((c + cp) % S1 != 0) {
          return false;
        }
      }
      int n0 = 0, m0 = 0;
      item(t, n0, m0);
      for (int m = 0; m < R; ++m)
        if (thread_of(n0 + R * m) / 64 != t / 64) return false;
    }
    return true;
  }
};
static_assert(FusedMap<8>::valid() && FusedMap<16>::valid() && FusedMap<32>::valid(), "fused layout");

template <class F>
constexpr bool fused_shape() {
  return F::R1 == F::R2 && F::R2 == F::R3 && F::NT == F::R1 * F::R1;
}

// Segment spectrum (packed half spectrum, natural order, [rows][M]) -> the
// fused layout: row position k2 NT + t holds bin col(t) + S1 k2.
template <typename T, int R>
__global__ __launch_bounds__(256) void fused_permute_kernel(const cx<T>* __restrict__ in, cx<T>* __restrict__ out) {
  constexpr int NT = R * R, M = R * R * R;
  const uint32_t pos = blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= uint32_t(M)) return;
  const uint32_t k2 = pos / NT, t = pos % NT;
  const uint64_t row = blockIdx.y;
  out[row * M + pos] = in[row * M + uint32_t(FusedMap<R>::col(int(t))) + uint32_t(NT) * k2];
}

// In-register pruned DFT: v[0..R) on entry holds x_r for r < NZ (the rest are
// zero and not read); on exit V[k] = sum_{r<NZ} x_r exp(DIR 2 pi i r k / R).
// With Q = R / NZ and k = a Q + b: V[a Q + b] = DFT_NZ(x_r w^{b r})[a],
// w = exp(DIR 2 pi i / R).
template <int R, int NZ, int DIR, typename T>
__device__ __forceinline__ void dft_pruned(cx<T>* v) {
  static_assert(NZ >= 1 && R % NZ == 0, "pruned size");
  if constexpr (NZ == R) {
    dft<R, DIR, T>(v);
  } else {
    constexpr int Q = R / NZ;
    cx<T> x[NZ];
#pragma unroll
    for (int r = 0; r < NZ; ++r) x[r] = v[r];
    static_for<Q>([&](auto bc) {
      constexpr int b = decltype(bc)::value;
      cx<T> u[NZ];
      static_for<NZ>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        u[r] = rot<b * r, R, DIR>(x[r]);
      });
      dft<NZ, DIR, T>(u);
#pragma unroll
      for (int a = 0; a < NZ; ++a) v[a * Q + b] = u[a];
    });
  }
}

// Forward transform of one template on chip (DIR = -1), leaving Z_k, k = col(t) + S1 k2,
// in v[k2].  rows: the first NZ input rows (k2 < NZ) of thread t's column t.  tw2s:
// the LDS copy of the pass-2 table where tw2_in_lds<F>() (ordered before use by
// exchange 1's barriers), else the table itself.
template <class F, int NZ, typename T>
__device__ __forceinline__ void fused_forward(cx<T>* v, T* lds, const cx<T>* __restrict__ tw1,
                                              const cx<T>* tw2s, int t, int n0, int m0) {
  constexpr int R = F::R1;
  const uint32_t colf[1] = {uint32_t(t)};
  {  // pass 1: pruned DFT over the rows, then w_M^(-n0 col)
    const Anchors<R, T> an = twiddle_load<R, T>(tw1, F::S1, colf[0]);
    dft_pruned<R, NZ, -1, T>(v);
    twiddle_apply<R, -1, T>(v, an);
    sched_fence();
  }
  // pass-2 item: (n0, j1) with j1 = m0 (the thread's own pass-3 index); table
  // anchors are requested before the exchange, whose barriers hide the wait
  Anchors<R, T> an2{};
  if constexpr (!tw2_in_lds<F>()) an2 = twiddle_load<R, T>(tw2s, F::R3, uint32_t(m0));
  auto ex1_read = [&](int pl) {
#pragma unroll
    for (int j2 = 0; j2 < R; ++j2) {
      const T a = lds[n0 * F::EX1_ROW + m0 + R * j2];
      if (pl == 0) v[j2].x = a;
      else v[j2].y = a;
    }
  };
  fft3_ex1_write<F, 0>(v, lds, colf);
  lds_barrier();
  ex1_read(0);
  lds_barrier();
  fft3_ex1_write<F, 1>(v, lds, colf);
  lds_barrier();
  ex1_read(1);
  lds_barrier();
  dft<R, -1, T>(v);
  sched_fence();
  if constexpr (tw2_in_lds<F>()) {
    twiddle_apply_lds<R, -1, T>(v, tw2s, F::R3, uint32_t(m0));
  } else {
    twiddle_apply<R, -1, T>(v, an2);
  }
  sched_fence();
  // exchange 2 inside the n0 group (one wave): write [m][j1 = m0], read [m0][j1]
  T* grp = lds + n0 * R * (R + 1);
#pragma unroll
  for (int pl = 0; pl < 2; ++pl) {
#pragma unroll
    for (int m = 0; m < R; ++m) grp[m * (R + 1) + m0] = pl == 0 ? v[m].x : v[m].y;
    wave_lds_fence();
#pragma unroll
    for (int j1 = 0; j1 < R; ++j1) {
      const T a = grp[m0 * (R + 1) + j1];
      if (pl == 0) v[j1].x = a;
      else v[j1].y = a;
    }
    wave_lds_fence();
  }
  dft<R, -1, T>(v);
  // the transform completes before the unpack starts: interleaving the two
  // keeps the DFT's temporaries and the unpack's partners live together
#pragma unroll
  for (int i = 0; i < R; ++i) pin(v[i]);
  sched_fence();
}

// Unpack Z (complex FFT of z_n = w_{2n} + i w_{2n+1}) into the packed real
// spectrum of w, scaled by sc, in place:
//   E_k = (Z_k + conj Z_{M-k}) / 2,  O_k = -i (Z_k - conj Z_{M-k}) / 2,
//   W_k = E_k + s_k O_k,  s_k = exp(-2 pi i k / N);  slot 0 of column 0:
//   (W_0, W_M) = (Re Z_0 + Im Z_0, Re Z_0 - Im Z_0).
// E_{M-k} = conj E_k, O_{M-k} = conj O_k and s_{M-k} = -conj s_k give
// W_{M-k} = conj(E_k - s_k O_k): one lane forms both values of a pair
// (mirror_pairs; partners as in the repack, columns 0 and S1/2 within their
// own lane, bin M/2 of column 0 with itself: W = sc conj Z).
// bu = exp(2 pi i col / N).
template <class F, typename T>
__device__ __forceinline__ void fused_unpack(cx<T>* v, const cx<T>& bu, T sc, int t) {
  static_assert(F::C1 == 1, "one column per thread");
  const T hs = T(0.5) * sc;
  const cx<T> z0 = v[0];  // lane 0 of wave 0: Z_0
  mirror_pairs<F, true, T>(
      v, t, cx<T>{T(0), T(0)}, [](int) {},
      [&](int, auto r1c, const cx<T>& A, const cx<T>& bp, cx<T>& wa, cx<T>& wb) {
        constexpr int r1 = decltype(r1c)::value;
        const cx<T> e = {A.x + bp.x, A.y - bp.y};   // 2 E_k
        const cx<T> od = {A.y + bp.y, bp.x - A.x};  // 2 O_k
        const cx<T> so = cmulc(rot<r1, 2 * F::R1, +1>(bu), od);
        wa = cx<T>{(e.x + so.x) * hs, (e.y + so.y) * hs};
        wb = cx<T>{(e.x - so.x) * hs, (so.y - e.y) * hs};  // W_{M-k}
      },
      [&](const cx<T>& m) { return cx<T>{m.x * sc, -m.y * sc}; });
  if (__builtin_amdgcn_readfirstlane(t) < 64)
    v[0] = lane_sel(1ull, v[0], cx<T>{(z0.x + z0.y) * sc, (z0.x - z0.y) * sc});
  pin(v[0]);
}

// Product with the segment spectrum (fused layout, loads G registers ahead) and the
// FP64 Parseval sum: v <- C = conj(W) Y; returns C_M (real) of column 0 in cM.
template <class F, int G, typename T>
__device__ __forceinline__ void fused_product(cx<T>* v, double& acc, T& cM, const rsrc_t& rY, int t, bool dc) {
  constexpr int R = F::R1, NG = R / G;
  constexpr uint32_t SY = sizeof(cx<T>);
  static_assert(R % G == 0, "group size");
  cx<T> ly[2][G];
  auto issue = [&](int g, int buf) {
#pragma unroll
    for (int e = 0; e < G; ++e)
      ly[buf][e] = buf_load<cx<T>>(rY, uint32_t(t) * SY, uint32_t((g * G + e) * F::NT) * SY);
  };
  issue(0, 0);
  cM = T(0);
  static_for<NG>([&](auto gc) {
    constexpr int g = decltype(gc)::value;
    if constexpr (g + 1 < NG) issue(g + 1, (g + 1) & 1);
    static_for<G>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      constexpr int k2 = g * G + e;
      cx<T> wk = v[k2], yk = ly[g & 1][e];
      if constexpr (k2 == 0) {
        cM = dc ? wk.y * yk.y : T(0);
        wk.y = dc ? T(0) : wk.y;
        yk.y = dc ? T(0) : yk.y;
      }
      const cx<T> ck = cmulc(wk, yk);
      double pk = 2.0 * (double(ck.x) * double(ck.x) + double(ck.y) * double(ck.y));
      if constexpr (k2 == 0) {
        const double pdc = double(ck.x) * double(ck.x) + double(cM) * double(cM);
        pk = dc ? pdc : pk;
      }
      acc += pk;
      v[k2] = ck;
      pin(v[k2]);
    });
    pin(acc);
    sched_fence();
  });
}

// One workgroup per (template j, spectrum row) in the order of tile_map, as
// corr_kernel (arguments alike), with the template synthesised on chip:
//   f0 / fdot / len [K]: grid parameters of templates j0.., norm [K] their
//   unit-norm factors, fs, taper, sym (time-symmetric chirps); yspec: the
//   segment spectra in the fused layout.
template <typename T, class F, bool DENSE, int G, int NZ>
__global__ __launch_bounds__(F::NT) void corr_fused_kernel(
    const cx<T>* __restrict__ yspec, const uint32_t* __restrict__ seg_ids, const cx<T>* __restrict__ tw_u,
    const cx<T>* __restrict__ tw1, const cx<T>* __restrict__ tw2, const double* __restrict__ f0,
    const double* __restrict__ fdot, const uint32_t* __restrict__ len, const float* __restrict__ norm, double fs,
    int taper, int sym, uint32_t K, uint32_t n_rows, uint32_t tile, double kappa, double* __restrict__ sigma_out,
    tail_rec_t<T>* __restrict__ tails, unsigned long long* __restrict__ counter, uint64_t cap,
    unsigned long long* __restrict__ proj, const uint64_t* __restrict__ proj_off, double kappa_hi,
    T* __restrict__ rho_dense, uint32_t j0, uint32_t k_total, uint32_t row0) {
  static_assert(fused_shape<F>(), "fused kernels need a cubic transform with one column per thread");
  constexpr int R = F::R1, M = F::M;
  constexpr double N = 2.0 * M;
  __shared__ T lds[F::LDS_ELEMS];
  __shared__ double red[F::NW];
  constexpr bool TWL = tw2_in_lds<F>();
  __shared__ cx<T> tw2s[TWL ? F::R2 * F::R3 : 1];
  const int t = threadIdx.x;
  uint32_t j, row;
  if (!tile_map(blockIdx.x, K, n_rows, tile, j, row)) return;
  if constexpr (TWL) fft3_tw2_stage<F>(tw2s, tw2, t);
  const uint32_t s = __builtin_amdgcn_readfirstlane(seg_ids ? seg_ids[row] : row0 + row);
  const uint32_t jg = j0 + j;
  int n0 = 0, m0 = 0;
  FusedMap<R>::item(t, n0, m0);
  const uint32_t cols[1] = {uint32_t(n0 + R * m0)};
  cx<T> bu = tw_u[cols[0]];  // exp(2 pi i col / N), for the unpack and the repack

  // 1. synthesis: z_k = (w_{2k}, w_{2k+1}), k = t + S1 r, rows r < NZ
  cx<T> v[F::P];
  {
    const double pf0 = f0[j], pfd = fdot[j];
    const int L = int(len[j]);
#pragma unroll
    for (int r = 0; r < NZ; ++r) {
      const int kk = t + F::S1 * r;
      double a = 0.0, b = 0.0;
      if (2 * kk < L) {
        a = chirp_sample(2 * kk, L, pf0, pfd, fs, taper);
        b = chirp_sample(2 * kk + 1, L, pf0, pfd, fs, taper);
        if (sym) {
          a += chirp_sample(L - 1 - 2 * kk, L, pf0, pfd, fs, taper);
          if (2 * kk + 1 < L) b += chirp_sample(L - 2 - 2 * kk, L, pf0, pfd, fs, taper);
        }
      }
      v[r] = {T(a), T(b)};
      pin(v[r]);
      sched_fence();  // one row at a time: the FP64 synthesis of many rows at once spills
    }
  }
  // 2-3. forward transform and unpack into the unit-norm spectrum W
  fused_forward<F, NZ, T>(v, lds, tw1, TWL ? tw2s : tw2, t, n0, m0);
  fused_unpack<F, T>(v, bu, T(norm[j]), t);
  // opaque from here: otherwise the twiddles the unpack formed per register are
  // kept (spilled) across the product stage for the repack to reuse
  pin(bu);
  // 4. C = conj(W) Y, Parseval sum, repack
  double acc = 0.0;
  T cM = T(0);
  const rsrc_t rY = make_rsrc(yspec + uint64_t(row) * M, uint32_t(M) * uint32_t(sizeof(cx<T>)));
  fused_product<F, G, T>(v, acc, cM, rY, t, t == 0);
  repack_mirror<F, MAP_MIRROR, T>(v, cM, t, [&](int) { return bu; });
  lds_barrier();  // every wave has left the forward exchange before the inverse writes LDS
  // 5. inverse transform, sigma, threshold
  const double S = corr_ifft<F, T, 1, false, TWL>(v, lds, red, cols, tw1, TWL ? tw2s : tw2, t, acc);
  const double rootS = sqrt(S);
  if (t == 0 && sigma_out) sigma_out[uint64_t(s) * k_total + jg] = rootS / N;
  auto z = [&](int i) { return v[i]; };
  if constexpr (DENSE) {
    const rsrc_t rr = make_rsrc(rho_dense + (uint64_t(s) * k_total + jg) * uint64_t(2 * M),
                                uint32_t(M) * uint32_t(sizeof(cx<T>)));
    emit_dense<F, T>(z, 0u, N, rr, t);
  } else {
    const T thr = T(kappa * rootS);
    const T thr_hi = kappa_hi > 0.0 ? T(kappa_hi * rootS) : T(INFINITY);
    T mx = T(0);
#pragma unroll
    for (int i = 0; i < F::P; ++i) mx = fmax(mx, fmax(fabs(v[i].x), fabs(v[i].y)));
    const bool any = (mx > thr) && (rootS > 0.0);
    if (__ballot(any)) {
      unsigned long long* prow = proj ? proj + proj_off[row] : nullptr;
      emit_tails<F, T>(z, 0u, thr, thr_hi, any, s, jg, N, tails, counter, cap, prow, rootS, t);
    }
  }
}

}  // namespace bfs
