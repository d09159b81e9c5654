// Kernels of the matched-filter hot path (gfx950).
//
//  fwd_fft_kernel   forward real FFT of one real series per workgroup (a
//                   segment y, a grid chirp synthesised in place, or an
//                   explicit template), as a complex FFT of length M = N/2 on
//                   z_n = x_{2n} + i x_{2n+1}; writes the complex Z.
//  rfft_unpack_kernel   Z -> the half spectrum X_0..X_{N/2} in the packed
//                   layout [M] (X_0 real in .x of slot 0, X_{N/2} real in .y),
//                   scaled and converted to the storage type.
//  corr_kernel      one correlation (segment s, template j) per workgroup:
//                   C = conj(W) Y, FP64 Parseval sum, Hermitian repack,
//                   inverse complex FFT of length M on chip, |rho| > kappa
//                   sigma, ballot compaction of the tails.
#pragma once

#include "bfs_fft3.h"

namespace bfs {

struct tail_rec {
  uint32_t segment, template_id, lag, reserved;
  double rho;
};

enum Source : int { SRC_SAMPLES = 0, SRC_CHIRP = 1, SRC_EXPLICIT = 2 };

// ---------------------------------------------------------------- forward --
// x[m] for the chirp source: h[m] cos(2 pi frac(f0 t + fdot t^2 / 2)), t = m/fs,
// phase and taper in FP64 (the phase reaches ~10^4 cycles over a second).
__device__ __forceinline__ double chirp_sample(int m, int len, double f0, double fdot, double fs, int taper) {
  if (m >= len) return 0.0;
  const double t = double(m) / fs;
  const double cyc = f0 * t + 0.5 * fdot * t * t;
  const double frac = cyc - floor(cyc);
  double w = cospi(2.0 * frac);
  if (taper && len > 1) w *= 0.5 * (1.0 - cospi(2.0 * double(m) / double(len - 1)));
  return w;
}

template <typename T, class F, int SRC>
__global__ __launch_bounds__(F::NT) void fwd_fft_kernel(
    const void* __restrict__ src, uint64_t src_stride, uint32_t src_len,
    const double* __restrict__ f0, const double* __restrict__ fdot, const uint32_t* __restrict__ len,
    double fs, int taper, uint32_t first,
    const cx<T>* __restrict__ tw1, const cx<T>* __restrict__ tw2,
    cx<T>* __restrict__ out, double* __restrict__ inv_norm) {
  __shared__ T lds[F::LDS_ELEMS];
  __shared__ double red[F::NW];
  const int t = threadIdx.x;
  const uint32_t b = blockIdx.x;
  cx<T> v[F::P];
  double acc = 0.0;
  uint32_t cols[F::C1];
#pragma unroll
  for (int c = 0; c < F::C1; ++c) cols[c] = fft3_col<F, false>(t, c);

  // ---- load (source stage)
  if constexpr (SRC == SRC_CHIRP) {
    const uint32_t j = first + b;
    const double pf0 = f0[j], pfd = fdot[j];
    const int L = int(len[j]);
#pragma unroll
    for (int c = 0; c < F::C1; ++c) {
      const int col = int(cols[c]);
#pragma unroll
      for (int k2 = 0; k2 < F::R1; ++k2) {
        const int k = col + F::S1 * k2;
        double a = 0.0, bb = 0.0;
        if (2 * k < L) {
          a = chirp_sample(2 * k, L, pf0, pfd, fs, taper);
          bb = chirp_sample(2 * k + 1, L, pf0, pfd, fs, taper);
        }
        acc += a * a + bb * bb;
        v[c * F::R1 + k2] = {T(a), T(bb)};
        pin(v[c * F::R1 + k2]);
        if ((k2 & 1) == 1) {
          pin(acc);
          sched_fence();
        }
      }
    }
  } else if constexpr (SRC == SRC_EXPLICIT) {
    const double* x = static_cast<const double*>(src) + uint64_t(first + b) * src_stride;
#pragma unroll
    for (int c = 0; c < F::C1; ++c) {
      const int col = int(cols[c]);
#pragma unroll
      for (int k2 = 0; k2 < F::R1; ++k2) {
        const int k = col + F::S1 * k2;
        const double a = (uint32_t(2 * k) < src_len) ? x[2 * k] : 0.0;
        const double bb = (uint32_t(2 * k + 1) < src_len) ? x[2 * k + 1] : 0.0;
        v[c * F::R1 + k2] = {T(a), T(bb)};
      }
    }
  } else {
    const T* x = static_cast<const T*>(src) + uint64_t(b) * src_stride;
    const rsrc_t rx = make_rsrc(x, uint32_t(F::M) * uint32_t(sizeof(cx<T>)));
#pragma unroll
    for (int c = 0; c < F::C1; ++c) {
#pragma unroll
      for (int k2 = 0; k2 < F::R1; ++k2)
        v[c * F::R1 + k2] = buf_load<cx<T>>(rx, cols[c] * uint32_t(sizeof(cx<T>)), uint32_t(F::S1 * k2) * uint32_t(sizeof(cx<T>)));
    }
  }

  fft3_pass1<F, -1>(v, tw1, cols);
  if constexpr (SRC == SRC_CHIRP) {
    const double s = wave_sum(acc);
    if ((t & 63) == 0) red[t >> 6] = s;
  }
  fft3_ex1_write<F, 0>(v, lds, cols);
  __syncthreads();
  fft3_ex1_read<F, 0>(v, lds, t);
  __syncthreads();
  fft3_ex1_write<F, 1>(v, lds, cols);
  __syncthreads();
  fft3_ex1_read<F, 1>(v, lds, t);
  if constexpr (SRC == SRC_CHIRP) {
    if (t == 0) {
      double s = 0.0;
      for (int w = 0; w < F::NW; ++w) s += red[w];
      inv_norm[b] = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    }
  }
  __syncthreads();
  fft3_pass2<F, -1>(v, tw2, t);
  fft3_ex2<F>(v, lds, t);
  fft3_pass3<F, -1>(v);

  const rsrc_t ro = make_rsrc(out + uint64_t(b) * F::M, uint32_t(F::M) * uint32_t(sizeof(cx<T>)));
#pragma unroll
  for (int c = 0; c < F::C2; ++c) {
    const uint32_t n0m0 = uint32_t(fft3_out_index<F>(t, c, 0));
#pragma unroll
    for (int mp = 0; mp < F::R3; ++mp)
      buf_store(v[c * F::R3 + mp], ro, n0m0 * uint32_t(sizeof(cx<T>)), uint32_t(F::R1 * F::R2 * mp) * uint32_t(sizeof(cx<T>)));
  }
}

// Z (complex FFT of z_n = x_{2n} + i x_{2n+1}) -> packed half spectrum of x:
//   E_k = (Z_k + conj Z_{M-k}) / 2,  O_k = -i (Z_k - conj Z_{M-k}) / 2,
//   X_k = E_k + exp(-2 pi i k / N) O_k,   X_{M-k} = conj(E_k - exp(-2 pi i k/N) O_k),
//   X_0 = Re Z_0 + Im Z_0,  X_M = Re Z_0 - Im Z_0 (both real).
// tw_u holds exp(+2 pi i k / N); scale (per row, may be null) multiplies X.
// Z and out may alias (in-place): each thread reads both of its slots first.
template <typename T, typename TW>
__global__ __launch_bounds__(256) void rfft_unpack_kernel(const cx<T>* Z, TW* out,
                                                          const double* __restrict__ scale,
                                                          const cx<T>* __restrict__ tw_u, uint32_t M,
                                                          uint64_t out_row_offset) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t b = blockIdx.y;
  if (k > M / 2) return;
  const cx<T>* z = Z + uint64_t(b) * M;
  TW* o = out + (out_row_offset + b) * uint64_t(M);
  const T sc = scale ? T(scale[b]) : T(1);
  if (k == 0) {
    const cx<T> z0 = z[0];
    store_spec<TW, T>(o, 0, cx<T>{(z0.x + z0.y) * sc, (z0.x - z0.y) * sc});
    return;
  }
  const cx<T> zk = z[k], zp = z[M - k];
  const cx<T> e = {T(0.5) * (zk.x + zp.x), T(0.5) * (zk.y - zp.y)};
  // O = -i/2 (Zk - conj Zp) = 1/2 (Im(Zk) + Im(Zp), -(Re Zk - Re Zp))
  const cx<T> od = {T(0.5) * (zk.y + zp.y), T(-0.5) * (zk.x - zp.x)};
  const cx<T> w = conjg(tw_u[k]);
  const cx<T> wo = cmul(w, od);
  const cx<T> xk = {(e.x + wo.x) * sc, (e.y + wo.y) * sc};
  store_spec<TW, T>(o, k, xk);
  if (M - k != k) {
    const cx<T> xp = {(e.x - wo.x) * sc, -(e.y - wo.y) * sc};
    store_spec<TW, T>(o, M - k, xp);
  }
}

// Packed storage -> FP64 interleaved [rows][M+1][2] (diagnostics).
template <typename T, typename TW>
__global__ __launch_bounds__(256) void spectrum_export_kernel(const TW* __restrict__ in, double* __restrict__ out,
                                                              uint32_t M, uint64_t first_row) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t b = blockIdx.y;
  if (k > M) return;
  const TW* row = in + (first_row + b) * uint64_t(M);
  double* o = out + uint64_t(b) * (M + 1) * 2;
  double re, im;
  if (k == 0) {
    re = double(load_spec<TW, T>(row, 0).x);
    im = 0.0;
  } else if (k == M) {
    re = double(load_spec<TW, T>(row, 0).y);
    im = 0.0;
  } else {
    const cx<T> a = load_spec<TW, T>(row, k);
    re = double(a.x);
    im = double(a.y);
  }
  o[2 * k] = re;
  o[2 * k + 1] = im;
}

__global__ void fill_u64_kernel(unsigned long long* p, uint64_t n, unsigned long long v) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------ correlation --
// One workgroup per (template j = blockIdx.x, segment s = blockIdx.y).
//   bank  [K][M] packed template spectra (storage TW), Y [S][M] packed.
//   tw_u  exp(+2 pi i k / N), tw1/tw2 the FFT twiddles (see bfs_fft3.h).
// Repack of the Hermitian product C for the length-M inverse transform:
//   Z_k = (C_k + conj C_{M-k}) + i exp(+2 pi i k / N) (C_k - conj C_{M-k}),
// then z = IDFT_M(Z) gives z_n = N (rho_{2n} + i rho_{2n+1}).
// Parseval (FP64): S = |C_0|^2 + |C_M|^2 + 2 sum_{k=1}^{M-1} |C_k|^2,
// sigma = sqrt(S) / N and |rho| > kappa sigma  <=>  |z| > kappa sqrt(S).
template <typename T, typename TW, class F, bool DENSE>
__global__ __launch_bounds__(F::NT) void corr_kernel(
    const TW* __restrict__ bank, const cx<T>* __restrict__ yspec,
    const cx<T>* __restrict__ tw_u, const cx<T>* __restrict__ tw1, const cx<T>* __restrict__ tw2,
    uint32_t K, double kappa, double* __restrict__ sigma_out,
    tail_rec* __restrict__ tails, unsigned long long* __restrict__ counter, uint64_t cap,
    T* __restrict__ rho_dense) {
  constexpr int M = F::M;
  constexpr double N = 2.0 * M;
  __shared__ T lds[F::LDS_ELEMS];
  __shared__ double red[F::NW];
  const int t = threadIdx.x;
  const uint32_t j = blockIdx.x, s = blockIdx.y;
  const TW* W = bank + uint64_t(j) * M;
  const cx<T>* Y = yspec + uint64_t(s) * M;
  const rsrc_t rW = make_rsrc(W, uint32_t(M) * uint32_t(sizeof(TW)));
  const rsrc_t rY = make_rsrc(Y, uint32_t(M) * uint32_t(sizeof(cx<T>)));
  cx<T> v[F::P];
  double acc = 0.0;

  // ---- spectral product and Parseval partial sum.  Element (col, k2) is
  // k = col + S1 k2; slot 0 of thread 0 packs the real C_0 (x) and C_M (y).
  // The loads run one group of G elements ahead of the arithmetic.
  constexpr int G = 2, NG = F::R1 / G;
  static_assert(F::R1 % G == 0 && F::R1 % 2 == 0, "group size");
  constexpr uint32_t SW = sizeof(TW), SY = sizeof(cx<T>);
  uint32_t cols[F::C1];
#pragma unroll
  for (int c = 0; c < F::C1; ++c) cols[c] = fft3_col<F, true>(t, c);
  T cM = T(0);  // C_M of thread 0 (real)
#pragma unroll
  for (int c = 0; c < F::C1; ++c) {
    const uint32_t col = cols[c];
    const bool dc = (c == 0) && (col == 0u);
    TW lw[2][G];
    cx<T> ly[2][G];
    auto issue = [&](int g, int buf) {
#pragma unroll
      for (int e = 0; e < G; ++e) {
        const uint32_t k2 = uint32_t(g * G + e);
        lw[buf][e] = buf_load<TW>(rW, col * SW, uint32_t(F::S1) * k2 * SW);
        ly[buf][e] = buf_load<cx<T>>(rY, col * SY, uint32_t(F::S1) * k2 * SY);
      }
    };
    issue(0, 0);
    static_for<NG>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      if constexpr (g + 1 < NG) issue(g + 1, (g + 1) & 1);
      static_for<G>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        constexpr int k2 = g * G + e;
        cx<T> wk = load_spec<TW, T>(&lw[g & 1][e], 0), yk = ly[g & 1][e];
        if constexpr (k2 == 0) {
          if (c == 0) cM = dc ? wk.y * yk.y : T(0);
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
        v[c * F::R1 + k2] = ck;
        pin(v[c * F::R1 + k2]);
      });
      pin(acc);
      sched_fence();
    });
  }

  // ---- Hermitian repack for the length-M inverse transform:
  //   Z_k = (C_k + conj C_{M-k}) + i exp(+2 pi i k / N) (C_k - conj C_{M-k}).
  // The partner of (col, k2) is (S1 - col, R1-1-k2), held by lane l ^ 32 of the
  // same wave at register R1-1-k2 (mirror column map), so registers k2 and
  // R1-1-k2 swap halves as a pair.  Columns 0 and S1/2 (lanes 0 and 32 of
  // wave 0) pair inside their own column: col 0 with index (R1 - k2) mod R1
  // (k2 = 0 with C_M), col S1/2 with R1-1-k2.  exp(2 pi i k / N) =
  // exp(2 pi i col / N) exp(i pi k2 / R1): one table load per column.
  const int lane = t & 63;
  const bool wave0 = t < 64;
#pragma unroll
  for (int c = 0; c < F::C1; ++c) {
    const cx<T> bu = tw_u[cols[c]];
    cx<T> carry = {T(0), T(0)};
    static_for<F::R1 / 2>([&](auto kc) {
      constexpr int r1 = decltype(kc)::value;
      constexpr int r2 = F::R1 - 1 - r1;
      const cx<T> A = v[c * F::R1 + r1], B = v[c * F::R1 + r2];
      cx<T> PA, PB;
      partner_pair(A, B, PA, PB);
      if (c == 0 && wave0) {
        const cx<T> a0 = (r1 == 0) ? cx<T>{cM, T(0)} : carry;
        const cx<T> b0 = (r1 + 1 == r2) ? B : v[c * F::R1 + r1 + 1];
        PA.x = lane == 0 ? a0.x : (lane == 32 ? B.x : PA.x);
        PA.y = lane == 0 ? a0.y : (lane == 32 ? B.y : PA.y);
        PB.x = lane == 0 ? b0.x : (lane == 32 ? A.x : PB.x);
        PB.y = lane == 0 ? b0.y : (lane == 32 ? A.y : PB.y);
        carry = B;
      }
      auto repack = [&](const cx<T>& ck, const cx<T>& cp, const cx<T>& tk) {
        const cx<T> a = {ck.x + cp.x, ck.y - cp.y};   // C_k + conj C_{M-k}
        const cx<T> bq = {ck.x - cp.x, ck.y + cp.y};  // C_k - conj C_{M-k}
        const cx<T> u = cmul(tk, bq);
        return cx<T>{a.x - u.y, a.y + u.x};
      };
      v[c * F::R1 + r1] = repack(A, PA, rot<r1, 2 * F::R1, +1>(bu));
      v[c * F::R1 + r2] = repack(B, PB, rot<r2, 2 * F::R1, +1>(bu));
      pin(v[c * F::R1 + r1]);
      pin(v[c * F::R1 + r2]);
      if constexpr (r1 % 4 == 3) sched_fence();
    });
    sched_fence();
  }

  fft3_pass1<F, +1>(v, tw1, cols);
  {
    const double ws = wave_sum(acc);
    if ((t & 63) == 0) red[t >> 6] = ws;
  }
  fft3_ex1_write<F, 0>(v, lds, cols);
  __syncthreads();
  double S = 0.0;
#pragma unroll
  for (int w = 0; w < F::NW; ++w) S += red[w];
  fft3_ex1_read<F, 0>(v, lds, t);
  __syncthreads();
  fft3_ex1_write<F, 1>(v, lds, cols);
  __syncthreads();
  fft3_ex1_read<F, 1>(v, lds, t);
  __syncthreads();
  fft3_pass2<F, +1>(v, tw2, t);
  fft3_ex2<F>(v, lds, t);
  fft3_pass3<F, +1>(v);

  const double rootS = sqrt(S);
  if (t == 0 && sigma_out) sigma_out[uint64_t(s) * K + j] = rootS / N;

  if constexpr (DENSE) {
    const rsrc_t rr = make_rsrc(rho_dense + (uint64_t(s) * K + j) * uint64_t(2 * M), uint32_t(M) * uint32_t(sizeof(cx<T>)));
    const T inv = T(1.0 / N);
#pragma unroll
    for (int c = 0; c < F::C2; ++c) {
      const uint32_t n0m0 = uint32_t(fft3_out_index<F>(t, c, 0));
#pragma unroll
      for (int mp = 0; mp < F::R3; ++mp)
        buf_store(cx<T>{v[c * F::R3 + mp].x * inv, v[c * F::R3 + mp].y * inv}, rr, n0m0 * uint32_t(sizeof(cx<T>)),
                  uint32_t(F::R1 * F::R2 * mp) * uint32_t(sizeof(cx<T>)));
    }
  } else {
    // ---- threshold and compaction
    const T thr = T(kappa * rootS);
    T mx = T(0);
#pragma unroll
    for (int i = 0; i < F::P; ++i) mx = fmax(mx, fmax(fabs(v[i].x), fabs(v[i].y)));
    const bool any = (mx > thr) && (rootS > 0.0);
    if (__ballot(any)) {
      const int lane = t & 63;
      const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
      for (int c = 0; c < F::C2; ++c) {
#pragma unroll
        for (int mp = 0; mp < F::R3; ++mp) {
          const int n = fft3_out_index<F>(t, c, mp);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const T val = h ? v[c * F::R3 + mp].y : v[c * F::R3 + mp].x;
            const bool pred = any && (fabs(val) > thr);
            const uint64_t mask = __ballot(pred);
            if (mask) {
              const int leader = __ffsll((unsigned long long)mask) - 1;
              unsigned long long base = 0;
              if (lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
              base = __shfl(base, leader, 64);
              if (pred) {
                const uint64_t idx = base + __popcll(mask & below);
                if (idx < cap) {
                  tail_rec r;
                  r.segment = s;
                  r.template_id = j;
                  r.lag = uint32_t(2 * n + h);
                  r.reserved = 0;
                  r.rho = double(val) / N;
                  tails[idx] = r;
                }
              }
            }
          }
        }
      }
    }
  }
}

}  // namespace bfs
