// Kernels of the matched-filter hot path (gfx950).
//
//  fwd_fft_kernel   forward real FFT of one real series per workgroup (a
//                   segment y, a grid chirp synthesised in place, or an
//                   explicit template), as a complex FFT of length M = N/2 on
//                   z_n = x_{2n} + i x_{2n+1}; writes the complex Z.  At
//                   the split size (N = 2^17) a workgroup transforms the
//                   even or the odd samples of z (length M/2) and the unpack
//                   joins them.
//  rfft_unpack_kernel   Z -> the half spectrum X_0..X_{N/2} in the packed
//                   layout [M] (X_0 real in .x of slot 0, X_{N/2} real in .y),
//                   scaled and converted to the storage type.  Split rows
//                   hold the even bins first, then the odd bins.
//  corr_kernel      one correlation (segment s, template j) per workgroup:
//                   C = conj(W) Y, FP64 Parseval sum, Hermitian repack,
//                   inverse complex FFT of length M on chip, |rho| > kappa
//                   sigma, ballot compaction of the tails.
//  corr2_kernel     the same at the split size: the length-M inverse
//                   transform runs as two length-M/2 transforms (even and
//                   odd bins) joined by one radix-2 step.
#pragma once

#include "bfs_fft3.h"
#include "bfs_records.h"

namespace bfs {

enum Source : int { SRC_SAMPLES = 0, SRC_CHIRP = 1, SRC_EXPLICIT = 2, SRC_CHIRP_SYM = 3 };

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

// One forward transform per workgroup.  Segment items read their samples at
// the device address seg_ptr[item], or at src + item src_stride (elements of
// T) when seg_ptr is null; explicit templates at src + item src_stride.  With
// zs > 1 (segments only) a segment's length-(zs F::M) transform is split zs
// ways: workgroup b transforms the sub-sequence z_{r + zs m}, m < F::M, of
// segment b / zs (r = b mod zs), for fft_join_kernel to combine.  Without split, workgroup b transforms item b.  With split, workgroup b = 2 item + h transforms the
// samples z_{2n+h}, n < F::M (h = 0 even, 1 odd).  Spectra go to out + b F::M.
// zero (may be null): three counters the first workgroup clears (a job's tail
// counters, so the job needs no launch of its own for them).
// The chirp source writes the FP64 sum of x^2 over the samples it made to
// energy[b] (the unpack turns it into the unit-norm scale); SRC_CHIRP_SYM
// synthesises the chirp plus its time reversal, x[m] + x[L-1-m].
template <typename T, class F, int SRC>
__global__ __launch_bounds__(F::NT) void fwd_fft_kernel(
    const void* __restrict__ src, uint64_t src_stride, uint32_t src_len, const uint64_t* __restrict__ seg_ptr,
    const double* __restrict__ f0, const double* __restrict__ fdot, const uint32_t* __restrict__ len,
    double fs, int taper, uint32_t first,
    const cx<T>* __restrict__ tw1, const cx<T>* __restrict__ tw2,
    cx<T>* __restrict__ out, double* __restrict__ energy, int split, uint32_t zs,
    unsigned long long* __restrict__ zero) {
  __shared__ T lds[F::LDS_ELEMS];
  __shared__ double red[F::NW];
  const int t = threadIdx.x;
  const uint32_t b = blockIdx.x;
  if (zero && b == 0 && t < 3) zero[t] = 0ull;
  const uint32_t item = split ? (b >> 1) : (zs > 1 ? b / zs : b);
  const uint32_t half = split ? (b & 1u) : (zs > 1 ? b % zs : 0u);
  const uint32_t cs = split ? 2u : (zs > 1 ? zs : 1u);  // stride of z between the transform's samples
  cx<T> v[F::P];
  double acc = 0.0;
  uint32_t cols[F::C1];
#pragma unroll
  for (int c = 0; c < F::C1; ++c) cols[c] = fft3_col<F, MAP_PLAIN>(t, c);

  // ---- load (source stage): element (col, k2) is z_kk, kk = cs (col + S1 k2) + half
  if constexpr (SRC == SRC_CHIRP || SRC == SRC_CHIRP_SYM) {
    const uint32_t j = first + item;
    const double pf0 = f0[j], pfd = fdot[j];
    const int L = int(len[j]);
#pragma unroll
    for (int c = 0; c < F::C1; ++c) {
#pragma unroll
      for (int k2 = 0; k2 < F::R1; ++k2) {
        const int kk = int(cs * (cols[c] + uint32_t(F::S1 * k2)) + half);
        double a = 0.0, bb = 0.0;
        if (2 * kk < L) {
          a = chirp_sample(2 * kk, L, pf0, pfd, fs, taper);
          bb = chirp_sample(2 * kk + 1, L, pf0, pfd, fs, taper);
          if constexpr (SRC == SRC_CHIRP_SYM) {  // plus the time reversal: x[m] + x[L-1-m]
            a += chirp_sample(L - 1 - 2 * kk, L, pf0, pfd, fs, taper);
            if (2 * kk + 1 < L) bb += chirp_sample(L - 2 - 2 * kk, L, pf0, pfd, fs, taper);
          }
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
    const double* x = static_cast<const double*>(src) + uint64_t(first + item) * src_stride;
#pragma unroll
    for (int c = 0; c < F::C1; ++c) {
#pragma unroll
      for (int k2 = 0; k2 < F::R1; ++k2) {
        const uint32_t kk = cs * (cols[c] + uint32_t(F::S1 * k2)) + half;
        const double a = (2 * kk < src_len) ? x[2 * kk] : 0.0;
        const double bb = (2 * kk + 1 < src_len) ? x[2 * kk + 1] : 0.0;
        v[c * F::R1 + k2] = {T(a), T(bb)};
      }
    }
  } else {
    const T* x = seg_ptr ? reinterpret_cast<const T*>(uintptr_t(seg_ptr[item]))
                         : static_cast<const T*>(src) + uint64_t(item) * src_stride;
    constexpr uint32_t SC = sizeof(cx<T>);
    const rsrc_t rx = make_rsrc(x, cs * uint32_t(F::M) * SC);
#pragma unroll
    for (int c = 0; c < F::C1; ++c) {
#pragma unroll
      for (int k2 = 0; k2 < F::R1; ++k2)
        v[c * F::R1 + k2] = buf_load<cx<T>>(rx, (cs * cols[c] + half) * SC, cs * uint32_t(F::S1 * k2) * SC);
    }
  }

  fft3_pass1<F, -1>(v, tw1, cols);
  if constexpr (SRC == SRC_CHIRP || SRC == SRC_CHIRP_SYM) {
    const double s = wave_sum(acc);
    if ((t & 63) == 0) red[t >> 6] = s;
  }
  fft3_ex1_write<F, 0>(v, lds, cols);
  lds_barrier();
  fft3_ex1_read<F, 0>(v, lds, t);
  lds_barrier();
  fft3_ex1_write<F, 1>(v, lds, cols);
  lds_barrier();
  fft3_ex1_read<F, 1>(v, lds, t);
  if constexpr (SRC == SRC_CHIRP || SRC == SRC_CHIRP_SYM) {
    if (t == 0) {
      double s = 0.0;
      for (int w = 0; w < F::NW; ++w) s += red[w];
      energy[b] = s;
    }
  }
  lds_barrier();
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

// Position of bin k (0 < k < M) in a stored row: k itself, or for split rows
// k/2 for even k and M/2 + (k-1)/2 for odd k.  Slot 0 holds X_0 and X_M.
__device__ __forceinline__ uint32_t bin_pos(uint32_t k, uint32_t M, int split) {
  return split ? ((k & 1u) ? (M >> 1) + (k >> 1) : (k >> 1)) : k;
}

// Z (complex FFT of z_n = x_{2n} + i x_{2n+1}) -> packed half spectrum of x:
//   E_k = (Z_k + conj Z_{M-k}) / 2,  O_k = -i (Z_k - conj Z_{M-k}) / 2,
//   X_k = E_k + exp(-2 pi i k / N) O_k,   X_{M-k} = conj(E_k - exp(-2 pi i k/N) O_k),
//   X_0 = Re Z_0 + Im Z_0,  X_M = Re Z_0 - Im Z_0 (both real).
// tw_u holds exp(+2 pi i k / N), k < M.  A split item holds the transforms A
// (even samples) and B (odd samples) of length H = M/2, and
//   Z_k = A_{k mod H} + exp(-2 pi i k / M) B_{k mod H},  exp(2 pi i r / M) = tw_u[2 r].
// energy (may be null): per transform the sum of x^2; the scale is
// 1 / sqrt(total) (two partial sums per split item).
// Z and out may alias when not split (in place): each thread reads both of
// its slots before writing them.
template <typename T, typename TW>
__global__ __launch_bounds__(256) void rfft_unpack_kernel(const cx<T>* Z, TW* out, const double* __restrict__ energy,
                                                          const cx<T>* __restrict__ tw_u, uint32_t M,
                                                          uint64_t out_row_offset, int split) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t b = blockIdx.y;
  if (k > M / 2) return;
  const cx<T>* z = Z + uint64_t(b) * M;
  TW* o = out + (out_row_offset + b) * uint64_t(M);
  T sc = T(1);
  if (energy) {
    const double e = split ? energy[2 * b] + energy[2 * b + 1] : energy[b];
    sc = e > 0.0 ? T(1.0 / sqrt(e)) : T(0);
  }
  const uint32_t H = M >> 1;
  auto zat = [&](uint32_t kk) -> cx<T> {  // Z_kk, kk < M
    if (!split) return z[kk];
    const uint32_t r = kk < H ? kk : kk - H;
    cx<T> w = conjg(tw_u[2 * r]);
    if (kk >= H) w = {-w.x, -w.y};
    return cadd(z[r], cmul(w, z[H + r]));
  };
  if (k == 0) {
    const cx<T> z0 = zat(0);
    store_spec<TW, T>(o, 0, cx<T>{(z0.x + z0.y) * sc, (z0.x - z0.y) * sc});
    return;
  }
  const cx<T> zk = zat(k), zp = zat(M - k);
  const cx<T> e = {T(0.5) * (zk.x + zp.x), T(0.5) * (zk.y - zp.y)};
  // O = -i/2 (Zk - conj Zp) = 1/2 (Im(Zk) + Im(Zp), -(Re Zk - Re Zp))
  const cx<T> od = {T(0.5) * (zk.y + zp.y), T(-0.5) * (zk.x - zp.x)};
  const cx<T> w = conjg(tw_u[k]);
  const cx<T> wo = cmul(w, od);
  const cx<T> xk = {(e.x + wo.x) * sc, (e.y + wo.y) * sc};
  store_spec<TW, T>(o, bin_pos(k, M, split), xk);
  if (M - k != k) {
    const cx<T> xp = {(e.x - wo.x) * sc, -(e.y - wo.y) * sc};
    store_spec<TW, T>(o, bin_pos(M - k, M, split), xp);
  }
}

// Join of a transform split A ways by fwd_fft_kernel (zs = A): with the
// sub-transforms T_r[k2] = sum_m z_{r + A m} exp(-2 pi i m k2 / B), B = M / A,
//   Z_k = sum_{r<A} T_r[k mod B] exp(-2 pi i r k / M)
// (the twiddle of sub-transform r and the length-A DFT in one factor).  One
// thread per output k of one segment (blockIdx.y), so a segment's join spreads
// over M / 256 workgroups: A loads of T (coalesced over consecutive k), the
// twiddles from tw_u (exp(+2 pi i j / N), j < M: exp(-2 pi i m / M) is
// conj(tw_u[2m mod N]) or, past M, -conj(tw_u[2m mod N - M])), FMA sums.  M is a
// power of two; in and out are [segments][M] (in: A rows of B).
template <typename T, int A>
__global__ __launch_bounds__(256) void fft_join_kernel(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                       const cx<T>* __restrict__ tw_u, uint32_t M) {
  const uint32_t B = M / A;
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const uint64_t base = uint64_t(blockIdx.y) * M;
  const cx<T>* row = in + base + (k & (B - 1u));
  const uint32_t mask = 2u * M - 1u;
  // four partial sums (r mod 4): shorter FMA chains, smaller rounding growth
  constexpr int NA = A >= 4 ? 4 : A;
  cx<T> acc[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) acc[q] = {T(0), T(0)};
#pragma unroll
  for (int r = 0; r < A; ++r) {
    const cx<T> a = row[uint64_t(r) * B];
    const uint32_t e = (2u * uint32_t(r) * k) & mask;  // 2 (r k mod M)
    const cx<T> t = tw_u[e < M ? e : e - M];
    // w = exp(-2 pi i r k / M) = (t.x, -t.y), or (-t.x, t.y) past M
    const T wx = e < M ? t.x : -t.x, wy = e < M ? -t.y : t.y;
    cx<T>& c = acc[r % NA];
    c.x = fmad<T>(a.x, wx, fmad<T>(-a.y, wy, c.x));
    c.y = fmad<T>(a.x, wy, fmad<T>(a.y, wx, c.y));
  }
  cx<T> z = acc[0];
#pragma unroll
  for (int q = 1; q < NA; ++q) z = cadd(z, acc[q]);
  out[base + k] = z;
}

// Packed storage -> FP64 interleaved [rows][M+1][2] in natural bin order (diagnostics).
template <typename T, typename TW>
__global__ __launch_bounds__(256) void spectrum_export_kernel(const TW* __restrict__ in, double* __restrict__ out,
                                                              uint32_t M, uint64_t first_row, int split) {
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
    const cx<T> a = load_spec<TW, T>(row, bin_pos(k, M, split));
    re = double(a.x);
    im = double(a.y);
  }
  o[2 * k] = re;
  o[2 * k + 1] = im;
}

// ------------------------------------------------------------ correlation --
// Stage 1: spectral product, Parseval partial sum and Hermitian repack of one
// block of F::M bins, read from element row_off of the rows: the whole half
// spectrum (MAP_MIRROR, row_off 0), or at the split size the even bins
// (MAP_MIRROR, row_off 0) or the odd bins (MAP_MIRROR_ODD, row_off F::M).
//   C_k = conj(W_k) Y_k;  acc += 2 |C_k|^2 in FP64, and |C_0|^2 + |C_M|^2 for slot 0;
//   Z_k = (C_k + conj C_{M-k}) + i exp(+2 pi i k / N) (C_k - conj C_{M-k}).
// Element (col, k2) of the block is bin index k' = col + S1 k2.  Its partner
// (bin M-k) is held by lane l ^ 32 of the same wave at register R1-1-k2 under
// both mirror maps, so registers k2 and R1-1-k2 swap halves as a pair.  Under
// MAP_MIRROR columns 0 and S1/2 (lanes 0 and 32 of wave 0) pair inside their
// own column: col 0 with index (R1 - k2) mod R1 (k2 = 0 with C_M, packed in
// slot 0), col S1/2 with R1-1-k2; the odd map has no self-paired column.
// exp(2 pi i k / N) = tw_u[bu_mul col + bu_add] exp(i pi k2 / R1) (bin
// k = bu_mul k' + bu_add): one table load per column, a constant rotation per
// element.
struct NoHook {
  __device__ void operator()(int, int) const {}
};

// Every Hermitian pair (k, M - k) of a block whose column c and partner column
// S1 - c sit in lanes l and l ^ 32 of one wave (element (col, k2) pairs with
// lane l ^ 32's register R1-1-k2), in place.  pair(c, r1, A, Bp, a, b) forms
// from A (this lane's register r1 of column c) and Bp (its partner, register
// r2 = R1-1-r1 of lane l ^ 32) the new value a of A and b of Bp: lane l takes
// the pair (its own r1, lane l ^ 32's r2), fetches that register with a half
// swap and returns b with another; the pairs of lane l ^ 32 are the mirror
// image, so every pair is formed once.  col(c) runs before column c's pairs.
// FIX: columns 0 and S1/2 (lanes 0 and 32 of wave 0, column slot 0) pair
// inside their own lane: column S1/2 register r1 with r2, column 0 register r
// with R1 - r, register 0 with `last` (whose result is dropped) and register
// R1/2 with itself, whose new value is mid(its old value).  Wave 0 alone, in a
// uniform branch, first gives lane 0 lane 32's registers R1/2..R1-1 and lane 32
// lane 0's registers R1/2+1..R1-1 and `last`, so the common half swaps deliver
// each lane its own partners, and afterwards moves the results back.
template <class F, bool FIX, typename T, class Col, class Pair, class Mid>
__device__ __forceinline__ void mirror_pairs(cx<T>* v, int t, const cx<T>& last, Col&& col, Pair&& pair,
                                             Mid&& mid) {
  constexpr int H = F::R1 / 2;
  // wave-uniform (readfirstlane): the other waves branch around the fixups
  const bool wave0 = FIX && __builtin_amdgcn_readfirstlane(t) < 64;
  constexpr uint64_t L0 = 1ull, L32 = 1ull << 32;  // lane masks
  cx<T> vmid = {T(0), T(0)};  // register R1/2 as it came (lane 0's is used)
  if (wave0) {
    vmid = v[H];
    static_for<H>([&](auto kc) {
      constexpr int r2 = H + decltype(kc)::value;  // ascending: v[r2 + 1] still unchanged
      const cx<T> hr = halfrot(v[r2]);
      cx<T> hn;
      if constexpr (r2 + 1 < F::R1) {
        hn = halfrot(v[r2 + 1]);
      } else {
        hn = halfrot(last);
      }
      v[r2] = lane_sel(L32, lane_sel(L0, v[r2], hr), hn);
    });
  }
#pragma unroll
  for (int c = 0; c < F::C1; ++c) {
    col(c);
    static_for<H>([&](auto kc) {
      constexpr int r1 = decltype(kc)::value;
      constexpr int r2 = F::R1 - 1 - r1;
      cx<T> a, b;
      pair(c, kc, v[c * F::R1 + r1], halfrot(v[c * F::R1 + r2]), a, b);
      v[c * F::R1 + r1] = a;
      v[c * F::R1 + r2] = halfrot(b);
      pin(v[c * F::R1 + r1]);
      pin(v[c * F::R1 + r2]);
      if constexpr (r1 % 4 == 3) sched_fence();
    });
    sched_fence();
  }
  if (wave0) {
    // lane 0 now holds lane 32's results in R1/2..R1-1, lane 32 lane 0's
    // results of R1/2+1..R1-1 in R1/2..R1-2
    static_for<H>([&](auto kc) {
      constexpr int r2 = F::R1 - 1 - decltype(kc)::value;  // descending: v[r2 - 1] still unchanged
      const cx<T> h = halfrot(v[r2]);
      cx<T> l0;
      if constexpr (r2 == H) {
        l0 = mid(vmid);
      } else {
        l0 = halfrot(v[r2 - 1]);
      }
      v[r2] = lane_sel(L0, lane_sel(L32, v[r2], h), l0);
    });
  }
}

// The Hermitian repack of the product stage, in place on the registers of
// every column c (twiddle get_bu(c) = exp(2 pi i k / N) of the column's first
// bin, called once per column before its registers are repacked):
//   Z_k = (C_k + conj C_{M-k}) + i t_k (C_k - conj C_{M-k}),  t_k = exp(2 pi i k / N).
// With P = C_k + conj C_{M-k}, u = t_k (C_k - conj C_{M-k}) and
// t_{M-k} = -conj t_k, the partner's value is Z_{M-k} = conj(P - i u): one
// lane forms both from one twiddle (mirror_pairs).  Under MAP_MIRROR column 0
// pairs register 0 with C_M (cM, real) and its register R1/2 (bin M/2) with
// itself: Z = 2 conj C.
template <class F, int MAP, typename T, class BU>
__device__ __forceinline__ void repack_mirror(cx<T>* v, T cM, int t, BU&& get_bu) {
  cx<T> buc;
  mirror_pairs<F, MAP == MAP_MIRROR, T>(
      v, t, cx<T>{cM, T(0)}, [&](int c) { buc = get_bu(c); },
      [&](int, auto r1c, const cx<T>& A, const cx<T>& bp, cx<T>& za, cx<T>& zb) {
        constexpr int r1 = decltype(r1c)::value;
        const cx<T> tk = rot<r1, 2 * F::R1, +1>(buc);
        const cx<T> P = {A.x + bp.x, A.y - bp.y};
        const cx<T> u = cmul(tk, cx<T>{A.x - bp.x, A.y + bp.y});
        za = cx<T>{P.x - u.y, P.y + u.x};
        zb = cx<T>{P.x + u.y, u.x - P.y};  // Z_{M-k}
      },
      [&](const cx<T>& m) { return cx<T>{T(2) * m.x, T(-2) * m.y}; });
}

template <class F, int MAP, int G, typename T, typename TW, bool EARLY_BU = false, class Hook = NoHook>
__device__ __forceinline__ void corr_pre(cx<T>* v, double& acc, const uint32_t* cols, const rsrc_t& rW,
                                         const rsrc_t& rY, uint32_t row_off, const cx<T>* __restrict__ tw_u,
                                         uint32_t bu_mul, uint32_t bu_add, int t, Hook&& before_group = Hook{}) {
  // The loads run one group of G elements ahead of the arithmetic (the
  // autotuner picks G; deeper groups hide more latency, cost registers).
  // before_group(c, g) runs after group g + 1's loads are issued and before
  // group g's products overwrite registers c R1 + g G .. + G - 1.  EARLY_BU
  // requests the repack twiddles before the spectra (for callers that issue
  // stores in before_group: counters complete in issue order, so the
  // twiddles' wait then covers none of those stores).
  constexpr int NG = F::R1 / G;
  static_assert(G >= 1 && F::R1 % G == 0 && F::R1 % 2 == 0, "group size");
  constexpr uint32_t SW = sizeof(TW), SY = sizeof(cx<T>);
  constexpr bool HAS_DC = MAP == MAP_MIRROR;
  T cM = T(0);  // C_M of thread 0 (real)
  double ha = 0.0, hb = 0.0;  // sum of |C_k|^2 / 2 over this thread's bins
  cx<T> bu[F::C1];  // the repack twiddle of each column
  if constexpr (EARLY_BU) {
#pragma unroll
    for (int c = 0; c < F::C1; ++c) bu[c] = tw_u[bu_mul * cols[c] + bu_add];
  }
#pragma unroll
  for (int c = 0; c < F::C1; ++c) {
    const uint32_t col = cols[c];
    const bool dc = HAS_DC && (c == 0) && (col == 0u);
    TW lw[2][G];
    cx<T> ly[2][G];
    auto issue = [&](int g, int buf) {
#pragma unroll
      for (int e = 0; e < G; ++e) {
        const uint32_t k2 = uint32_t(g * G + e);
        lw[buf][e] = buf_load<TW>(rW, col * SW, (row_off + uint32_t(F::S1) * k2) * SW);
        ly[buf][e] = buf_load<cx<T>>(rY, col * SY, (row_off + uint32_t(F::S1) * k2) * SY);
      }
    };
    issue(0, 0);
    static_for<NG>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      if constexpr (g + 1 < NG) issue(g + 1, (g + 1) & 1);
      before_group(c, g);
      static_for<G>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        constexpr int k2 = g * G + e;
        cx<T> wk = load_spec<TW, T>(&lw[g & 1][e], 0), yk = ly[g & 1][e];
        if constexpr (HAS_DC && k2 == 0) {
          if (c == 0) cM = dc ? wk.y * yk.y : T(0);
          wk.y = dc ? T(0) : wk.y;
          yk.y = dc ? T(0) : yk.y;
        }
        const cx<T> ck = cmulc(wk, yk);
        // |C_k|^2 into two FP64 chains (products of FP32 values are exact in
        // FP64); the factor 2 is applied once at the end, so slot 0 of column
        // 0 adds half of |C_0|^2 + |C_M|^2
        const double dx = double(ck.x);
        if constexpr (HAS_DC && k2 == 0) {
          const double sc = dc ? 0.5 : 1.0;
          const double dy = dc ? double(cM) : double(ck.y);
          ha = fma(sc * dx, dx, ha);
          hb = fma(sc * dy, dy, hb);
        } else {
          const double dy = double(ck.y);
          ha = fma(dx, dx, ha);
          hb = fma(dy, dy, hb);
        }
        v[c * F::R1 + k2] = ck;
        pin(v[c * F::R1 + k2]);
      });
      pin(ha);
      pin(hb);
      sched_fence();
    });
  }
  acc += 2.0 * (ha + hb);

  repack_mirror<F, MAP, T>(v, cM, t, [&](int c) {
    if constexpr (!EARLY_BU) bu[c] = tw_u[bu_mul * cols[c] + bu_add];
    return bu[c];
  });
}

// Stage 2: inverse transform of length F::M on chip.  Returns the workgroup
// sum of every thread's acc, reduced in a fixed order (deterministic); with
// NACC = 2 also the sum of acc2 into *S2 (red then holds 2 F::NW doubles).
// PRE_BARRIER: a workgroup barrier before the first LDS write of the
// exchange, for callers that loop over correlations (every wave has then
// left the previous correlation's exchanges, whatever it did before).
// TW2S: tw2 is the LDS copy of the pass-2 table (fft3_tw2_stage).
template <class F, typename T, int NACC = 1, bool PRE_BARRIER = false, bool TW2S = false>
__device__ __forceinline__ double corr_ifft(cx<T>* v, T* lds, double* red, const uint32_t* cols,
                                            const cx<T>* __restrict__ tw1, const cx<T>* tw2, int t,
                                            double acc, double acc2 = 0.0, double* S2 = nullptr) {
  fft3_pass1<F, +1>(v, tw1, cols);
  {
    const double ws = wave_sum(acc);
    if ((t & 63) == 0) red[t >> 6] = ws;
    if constexpr (NACC == 2) {
      const double ws2 = wave_sum(acc2);
      if ((t & 63) == 0) red[F::NW + (t >> 6)] = ws2;
    }
  }
  Pass2Anchors<F, T> an2;
  if constexpr (!TW2S) an2 = fft3_pass2_load<F, T>(tw2, t);
  if constexpr (PRE_BARRIER) lds_barrier();
  fft3_ex1_write<F, 0>(v, lds, cols);
  lds_barrier();
  double S = 0.0;
#pragma unroll
  for (int w = 0; w < F::NW; ++w) S += red[w];
  // formed here: otherwise the compiler defers the additions to the sum's
  // use and keeps the NW partial sums live through the transform
  asm volatile("" : "+v"(S));
  if constexpr (NACC == 2) {
    double Sb = 0.0;
#pragma unroll
    for (int w = 0; w < F::NW; ++w) Sb += red[F::NW + w];
    asm volatile("" : "+v"(Sb));
    *S2 = Sb;
  }
  fft3_ex1_read<F, 0>(v, lds, t);
  lds_barrier();
  fft3_ex1_write<F, 1>(v, lds, cols);
  lds_barrier();
  fft3_ex1_read<F, 1>(v, lds, t);
  lds_barrier();
  if constexpr (TW2S) {
    fft3_pass2_tab<F, +1>(v, tw2, t);
  } else {
    fft3_pass2<F, +1>(v, an2);
  }
  fft3_ex2<F>(v, lds, t);
  fft3_pass3<F, +1>(v);
  return S;
}

// Stage 3, dense: z(i) is the value of register i (= N (rho_{2n} + i
// rho_{2n+1}) at n = n_off + output index of i); rho goes into the row.
template <class F, typename T, class Z>
__device__ __forceinline__ void emit_dense(Z&& z, uint32_t n_off, double N, const rsrc_t& rrow, int t) {
  const T inv = T(1.0 / N);
#pragma unroll
  for (int c = 0; c < F::C2; ++c) {
    const uint32_t n0m0 = uint32_t(fft3_out_index<F>(t, c, 0)) + n_off;
#pragma unroll
    for (int mp = 0; mp < F::R3; ++mp) {
      const cx<T> a = z(c * F::R3 + mp);
      buf_store(cx<T>{a.x * inv, a.y * inv}, rrow, n0m0 * uint32_t(sizeof(cx<T>)),
                uint32_t(F::R1 * F::R2 * mp) * uint32_t(sizeof(cx<T>)));
    }
  }
}

// Stage 3, threshold: keep thr < |z| < thr_hi (thr = kappa sqrt(S) in z units;
// thr_hi = kappa_hi sqrt(S) for a finite band, else +inf).  Called by the whole
// wave when some lane may hold a tail (any).  The wave counts its tails first,
// reserves them with one atomicAdd and a prefix sum of the per-lane counts,
// then every lane writes its own; records past cap are counted but not written.
// With prow set (per-lag max projection) a tail is not written to the list:
// it raises prow[lag] with atomicMax to the key
//   (float bits of |rho| / sigma) << 32 | (0x7fffffff - j) << 1 | (rho < 0),
// so the largest significance wins, equal significances go to the lowest
// template id, and the result does not depend on the order of the updates.
// rootS = sqrt(S) = N sigma, so |rho| / sigma = |z| / rootS.
template <class F, typename T, class Z>
__device__ __forceinline__ void emit_tails(Z&& z, uint32_t n_off, T thr, T thr_hi, bool any, uint32_t s, uint32_t j,
                                           double N, tail_rec_t<T>* __restrict__ tails,
                                           unsigned long long* __restrict__ counter, uint64_t cap,
                                           unsigned long long* __restrict__ prow, double rootS, int t) {
  const int lane = t & 63;
  auto is_tail = [&](T val) { return any && (fabs(val) > thr) && (fabs(val) < thr_hi); };
  uint32_t cnt = 0;
#pragma unroll
  for (int i = 0; i < F::P; ++i) {
    const cx<T> a = z(i);
    cnt += uint32_t(is_tail(a.x)) + uint32_t(is_tail(a.y));
  }
  uint32_t incl = cnt;  // inclusive prefix sum over the wave's lanes
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(incl, d, 64);
    if (lane >= d) incl += o;
  }
  const uint32_t total = __shfl(incl, 63, 64);
  if (total == 0) return;
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(counter, (unsigned long long)total);
  base = __shfl(base, 0, 64);
  if (cnt == 0) return;
  uint64_t idx = base + (incl - cnt);
#pragma unroll
  for (int c = 0; c < F::C2; ++c) {
#pragma unroll
    for (int mp = 0; mp < F::R3; ++mp) {
      const uint32_t n = uint32_t(fft3_out_index<F>(t, c, mp)) + n_off;
      const cx<T> a = z(c * F::R3 + mp);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        T val = h ? a.y : a.x;
        // Opaque to the compiler, so |val| is formed here, one value at a
        // time, and not hoisted for all 2 P values ahead of the loop (which
        // doubled the registers the kernel holds).
        asm volatile("" : "+v"(val));
        if (!is_tail(val)) continue;
        const uint32_t lag = 2 * n + uint32_t(h);
        if (prow) {
          const float snr = float(fabs(double(val)) / rootS);
          const unsigned long long key = (static_cast<unsigned long long>(__float_as_uint(snr)) << 32) |
                                         (static_cast<unsigned long long>(0x7fffffffu - j) << 1) |
                                         (val < T(0) ? 1ull : 0ull);
          atomicMax(prow + lag, key);
        } else if (idx < cap) {
          tail_rec_t<T> r{};
          r.segment = s;
          r.template_id = j;
          r.lag = lag;
          r.rho = decltype(r.rho)(double(val) / N);
          tails[idx] = r;
        }
        ++idx;
      }
    }
  }
}

// Workgroup order.  The hardware hands workgroups to the 8 XCDs round robin
// (b mod 8), so XCD x runs b = x, x + 8, x + 16, ...  Within an XCD the order
// is: tile of T segments, then template j = 8 jj + x, then the segment within
// the tile.  The T workgroups of one template run back to back on one XCD and
// read its bank row from that XCD's L2, while the tile's T segment spectra stay
// L2-resident as the tile sweeps the templates (T = 1: every template once per
// segment, the segment spectrum shared by all).  Returns false for the padding
// workgroups when K is not a multiple of 8.  Requires 1 <= T <= S.
__device__ __forceinline__ bool tile_map(uint32_t b, uint32_t K, uint32_t S, uint32_t T, uint32_t& j,
                                         uint32_t& row) {
  const uint32_t x = b & 7u, i = b >> 3;
  const uint32_t kx = (K + 7u - x) >> 3;  // templates with j = x (mod 8)
  if (i >= kx * S) return false;
  const uint32_t full = S / T, per_tile = kx * T;
  uint32_t jj, s;
  if (i < full * per_tile) {
    const uint32_t ti = i / per_tile, rem = i - ti * per_tile;
    jj = rem / T;
    s = ti * T + (rem - jj * T);
  } else {
    const uint32_t r = S - full * T, rem = i - full * per_tile;
    jj = rem / r;
    s = full * T + (rem - jj * r);
  }
  // the quotients above come out of VALU division code; readfirstlane marks
  // them wave-uniform so the buffer resources built from them stay scalar
  j = __builtin_amdgcn_readfirstlane(8u * jj + x);
  row = __builtin_amdgcn_readfirstlane(s);
  return true;
}

// One workgroup per (template j, spectrum row), in the order of tile_map over
// a 1-D grid of 8 ceil(K/8) n_rows workgroups.  A launch may cover a slice of
// the bank and of the rows (the host splits grids that would be too large):
//   bank  [K][M] packed template spectra (storage TW) of templates j0..j0+K-1,
//   yspec [n_rows][M] packed; row r is segment seg_ids[r] (or row0 + r), the
//   id used for sigma and tails; template ids are j0 + j, and sigma_out and
//   rho_dense are indexed by segment * k_total + template id;
//   proj (may be null): projection keys, row r's N lags at proj + proj_off[r].
//   tw_u  exp(+2 pi i k / N), tw1/tw2 the FFT twiddles (see bfs_fft3.h).
// z = IDFT_M(Z) gives z_n = N (rho_{2n} + i rho_{2n+1}); with
// S = |C_0|^2 + |C_M|^2 + 2 sum_{k=1}^{M-1} |C_k|^2 (FP64), sigma = sqrt(S)/N and
// |rho| > kappa sigma  <=>  |z| > kappa sqrt(S).
template <typename T, typename TW, class F, bool DENSE, int G>
__global__ __launch_bounds__(F::NT) void corr_kernel(
    const TW* __restrict__ bank, const cx<T>* __restrict__ yspec, const uint32_t* __restrict__ seg_ids,
    const cx<T>* __restrict__ tw_u, const cx<T>* __restrict__ tw1, const cx<T>* __restrict__ tw2,
    uint32_t K, uint32_t n_rows, uint32_t tile, double kappa, double* __restrict__ sigma_out,
    tail_rec_t<T>* __restrict__ tails, unsigned long long* __restrict__ counter, uint64_t cap,
    unsigned long long* __restrict__ proj, const uint64_t* __restrict__ proj_off, double kappa_hi,
    T* __restrict__ rho_dense, uint32_t j0, uint32_t k_total, uint32_t row0) {
  constexpr int M = F::M;
  constexpr double N = 2.0 * M;
  constexpr bool TWL = tw2_in_lds<F>();
  __shared__ T lds[F::LDS_ELEMS];
  __shared__ double red[F::NW];
  __shared__ cx<T> tw2s[TWL ? F::R2 * F::R3 : 1];
  const int t = threadIdx.x;
  uint32_t j, row;
  if (!tile_map(blockIdx.x, K, n_rows, tile, j, row)) return;
  if constexpr (TWL) fft3_tw2_stage<F>(tw2s, tw2, t);
  const uint32_t s = __builtin_amdgcn_readfirstlane(seg_ids ? seg_ids[row] : row0 + row);
  const uint32_t jg = j0 + j;  // template id in the whole bank
  const rsrc_t rW = make_rsrc(bank + uint64_t(j) * M, uint32_t(M) * uint32_t(sizeof(TW)));
  const rsrc_t rY = make_rsrc(yspec + uint64_t(row) * M, uint32_t(M) * uint32_t(sizeof(cx<T>)));
  cx<T> v[F::P];
  double acc = 0.0;
  uint32_t cols[F::C1];
#pragma unroll
  for (int c = 0; c < F::C1; ++c) cols[c] = fft3_col<F, MAP_MIRROR>(t, c);
  // 32 points per thread: these kernels hold 4 waves per SIMD whatever their
  // register count below 128, so the early twiddle request is free
  corr_pre<F, MAP_MIRROR, G, T, TW, (F::P >= 32)>(v, acc, cols, rW, rY, 0u, tw_u, 1u, 0u, t);
  const double S = corr_ifft<F, T, 1, false, TWL>(v, lds, red, cols, tw1, TWL ? tw2s : tw2, t, acc);
  const double rootS = sqrt(S);
  if (t == 0 && sigma_out) sigma_out[uint64_t(s) * k_total + jg] = rootS / N;
  auto z = [&](int i) { return v[i]; };
  if constexpr (DENSE) {
    const rsrc_t rr = make_rsrc(rho_dense + (uint64_t(s) * k_total + jg) * uint64_t(2 * M), uint32_t(M) * uint32_t(sizeof(cx<T>)));
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

// One correlation (template j of the launch's bank slice, spectrum row `row`)
// by one workgroup of corr_loop_kernel: corr_kernel's stages, with the barrier
// before the exchange that looping needs; tw2 is the workgroup's LDS copy of
// the pass-2 twiddle table where tw2_in_lds<F>().  (corr_kernel keeps its own
// copy of this sequence: sharing the function changed its register schedule.)
template <typename T, typename TW, class F, bool DENSE, int G>
__device__ __forceinline__ void corr_item(
    uint32_t j, uint32_t row, T* lds, double* red, const TW* __restrict__ bank, const cx<T>* __restrict__ yspec,
    const uint32_t* __restrict__ seg_ids, const cx<T>* __restrict__ tw_u, const cx<T>* __restrict__ tw1,
    const cx<T>* __restrict__ tw2, double kappa, double* __restrict__ sigma_out, tail_rec_t<T>* __restrict__ tails,
    unsigned long long* __restrict__ counter, uint64_t cap, unsigned long long* __restrict__ proj,
    const uint64_t* __restrict__ proj_off, double kappa_hi, T* __restrict__ rho_dense, uint32_t j0, uint32_t k_total,
    uint32_t row0, int t) {
  constexpr int M = F::M;
  constexpr double N = 2.0 * M;
  const uint32_t s = __builtin_amdgcn_readfirstlane(seg_ids ? seg_ids[row] : row0 + row);
  const uint32_t jg = j0 + j;  // template id in the whole bank
  const rsrc_t rW = make_rsrc(bank + uint64_t(j) * M, uint32_t(M) * uint32_t(sizeof(TW)));
  const rsrc_t rY = make_rsrc(yspec + uint64_t(row) * M, uint32_t(M) * uint32_t(sizeof(cx<T>)));
  cx<T> v[F::P];
  double acc = 0.0;
  uint32_t cols[F::C1];
#pragma unroll
  for (int c = 0; c < F::C1; ++c) cols[c] = fft3_col<F, MAP_MIRROR>(t, c);
  // 32 points per thread: these kernels hold 4 waves per SIMD whatever their
  // register count below 128, so the early twiddle request is free
  corr_pre<F, MAP_MIRROR, G, T, TW, (F::P >= 32)>(v, acc, cols, rW, rY, 0u, tw_u, 1u, 0u, t);
  const double S = corr_ifft<F, T, 1, true, tw2_in_lds<F>()>(v, lds, red, cols, tw1, tw2, t, acc);
  const double rootS = sqrt(S);
  if (t == 0 && sigma_out) sigma_out[uint64_t(s) * k_total + jg] = rootS / N;
  auto z = [&](int i) { return v[i]; };
  if constexpr (DENSE) {
    const rsrc_t rr = make_rsrc(rho_dense + (uint64_t(s) * k_total + jg) * uint64_t(2 * M), uint32_t(M) * uint32_t(sizeof(cx<T>)));
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

// The same correlations with fewer workgroups, each looping over items
// b, b + gridDim.x, b + 2 gridDim.x, ... < n_items of the tile_map order (a
// multiple of 8 workgroups keeps every item on the XCD tile_map gives it).
// The waves of a workgroup need not finish one correlation together: a wave
// done early loads and multiplies the next correlation's spectra while the
// others finish the last one, up to the barrier before the next exchange, so
// the spectrum latency at the start of a correlation and the spread of its
// waves at the end overlap.
template <typename T, typename TW, class F, bool DENSE, int G>
__global__ __launch_bounds__(F::NT) void corr_loop_kernel(
    const TW* __restrict__ bank, const cx<T>* __restrict__ yspec, const uint32_t* __restrict__ seg_ids,
    const cx<T>* __restrict__ tw_u, const cx<T>* __restrict__ tw1, const cx<T>* __restrict__ tw2,
    uint32_t K, uint32_t n_rows, uint32_t tile, double kappa, double* __restrict__ sigma_out,
    tail_rec_t<T>* __restrict__ tails, unsigned long long* __restrict__ counter, uint64_t cap,
    unsigned long long* __restrict__ proj, const uint64_t* __restrict__ proj_off, double kappa_hi,
    T* __restrict__ rho_dense, uint32_t j0, uint32_t k_total, uint32_t row0, uint32_t n_items) {
  constexpr bool TWL = tw2_in_lds<F>();
  __shared__ T lds[F::LDS_ELEMS];
  __shared__ double red[F::NW];
  __shared__ cx<T> tw2s[TWL ? F::R2 * F::R3 : 1];
  if constexpr (TWL) fft3_tw2_stage<F>(tw2s, tw2, int(threadIdx.x));
  for (uint32_t i = blockIdx.x; i < n_items; i += gridDim.x) {
    uint32_t j, row;
    if (!tile_map(i, K, n_rows, tile, j, row)) continue;
    // an opaque copy of the thread index per item: the lane addresses derived from it
    // are formed where used, not hoisted out of the loop and kept (spilled) across it
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    corr_item<T, TW, F, DENSE, G>(j, row, lds, red, bank, yspec, seg_ids, tw_u, tw1, TWL ? tw2s : tw2, kappa, sigma_out,
                                        tails, counter, cap, proj, proj_off, kappa_hi, rho_dense, j0, k_total, row0, t);
  }
}

// Split size: M = 2 H, H = F::M.  The even bins (row elements [0, H)) and
// the odd bins ([H, M)) are each repacked and inverse-transformed at length
// H, giving E and O; then
//   z_n = E_n + exp(2 pi i n / M) O_n,   z_{n+H} = E_n - exp(2 pi i n / M) O_n.
// E waits in per-thread scratch memory while the odd half runs (each thread
// reads back only what it stored).  exp(2 pi i n / M) for
// n = n0 + R1 m0 + R1 R2 m' is tw_u[2 (n0 + R1 m0)] exp(i pi m' / R3).
template <typename T, typename TW, class F, bool DENSE, int G>
__global__ __launch_bounds__(F::NT) void corr2_kernel(
    const TW* __restrict__ bank, const cx<T>* __restrict__ yspec, const uint32_t* __restrict__ seg_ids,
    const cx<T>* __restrict__ tw_u, const cx<T>* __restrict__ tw1, const cx<T>* __restrict__ tw2,
    uint32_t K, uint32_t n_rows, uint32_t tile, double kappa, double* __restrict__ sigma_out,
    tail_rec_t<T>* __restrict__ tails, unsigned long long* __restrict__ counter, uint64_t cap,
    unsigned long long* __restrict__ proj, const uint64_t* __restrict__ proj_off, double kappa_hi,
    T* __restrict__ rho_dense, uint32_t j0, uint32_t k_total, uint32_t row0) {
  constexpr int H = F::M, M = 2 * H;
  constexpr double N = 2.0 * M;
  __shared__ T lds[F::LDS_ELEMS];
  __shared__ double red[F::NW];
  const int t = threadIdx.x;
  uint32_t j, row;
  if (!tile_map(blockIdx.x, K, n_rows, tile, j, row)) return;
  const uint32_t s = __builtin_amdgcn_readfirstlane(seg_ids ? seg_ids[row] : row0 + row);
  const uint32_t jg = j0 + j;  // template id in the whole bank
  const rsrc_t rW = make_rsrc(bank + uint64_t(j) * M, uint32_t(M) * uint32_t(sizeof(TW)));
  const rsrc_t rY = make_rsrc(yspec + uint64_t(row) * M, uint32_t(M) * uint32_t(sizeof(cx<T>)));
  cx<T> v[F::P];
  // E waits in per-thread scratch memory: the array's address escapes into
  // an empty asm statement, so it stays in memory (ordinary cached scratch
  // accesses) instead of being promoted to registers.  The stores go out one
  // load group at a time inside the odd half's product stage, each after the
  // next group's loads are issued: vector-memory counters complete in issue
  // order, so no wait for an odd-half load ever covers an E store issued
  // after it, and the stores drain under the odd half's arithmetic.
  cx<T> e[F::P];
  asm volatile("" : : "v"(e) : "memory");

  double acc = 0.0;
  uint32_t cols[F::C1];
#pragma unroll
  for (int c = 0; c < F::C1; ++c) cols[c] = fft3_col<F, MAP_MIRROR>(t, c);
  corr_pre<F, MAP_MIRROR, G, T, TW, true>(v, acc, cols, rW, rY, 0u, tw_u, 2u, 0u, t);
  const double S0 = corr_ifft<F>(v, lds, red, cols, tw1, tw2, t, acc);

  // The odd half derives its lane addresses from an opaque copy of the thread
  // index, so nothing computed for the even half is kept (spilled) for reuse.
  int to = t;
  asm volatile("" : "+v"(to));
  acc = 0.0;
#pragma unroll
  for (int c = 0; c < F::C1; ++c) cols[c] = fft3_col<F, MAP_MIRROR_ODD>(to, c);
  corr_pre<F, MAP_MIRROR_ODD, G, T, TW, true>(v, acc, cols, rW, rY, uint32_t(H), tw_u, 2u, 1u, to, [&](int c, int g) {
#pragma unroll
    for (int k = 0; k < G; ++k) e[c * F::R1 + g * G + k] = v[c * F::R1 + g * G + k];
    asm volatile("" ::: "memory");
  });
  asm volatile("" : : "v"(e) : "memory");
  lds_barrier();  // every wave is done with the even half's LDS before the odd half writes it
  const double S = S0 + corr_ifft<F>(v, lds, red, cols, tw1, tw2, to, acc);
  const double rootS = sqrt(S);
  if (t == 0 && sigma_out) sigma_out[uint64_t(s) * k_total + jg] = rootS / N;

  // v <- exp(2 pi i n / M) O_n
#pragma unroll
  for (int c = 0; c < F::C2; ++c) {
    const cx<T> bc = tw_u[2 * fft3_out_index<F>(to, c, 0)];
    static_for<F::R3>([&](auto mc) {
      constexpr int mp = decltype(mc)::value;
      v[c * F::R3 + mp] = cmul(rot<mp, 2 * F::R3, +1>(bc), v[c * F::R3 + mp]);
    });
  }
  auto z_lo = [&](int i) { return cadd(e[i], v[i]); };
  auto z_hi = [&](int i) { return csub(e[i], v[i]); };
  if constexpr (DENSE) {
    const rsrc_t rr = make_rsrc(rho_dense + (uint64_t(s) * k_total + jg) * uint64_t(2 * M), uint32_t(M) * uint32_t(sizeof(cx<T>)));
    emit_dense<F, T>(z_lo, 0u, N, rr, t);
    emit_dense<F, T>(z_hi, uint32_t(H), N, rr, t);
  } else {
    const T thr = T(kappa * rootS);
    const T thr_hi = kappa_hi > 0.0 ? T(kappa_hi * rootS) : T(INFINITY);
    T mx = T(0);
#pragma unroll
    for (int i = 0; i < F::P; ++i) {
      const T a = e[i].x, b = e[i].y;
      mx = fmax(mx, fmax(fmax(fabs(a + v[i].x), fabs(b + v[i].y)), fmax(fabs(a - v[i].x), fabs(b - v[i].y))));
    }
    const bool any = (mx > thr) && (rootS > 0.0);
    if (__ballot(any)) {
      unsigned long long* prow = proj ? proj + proj_off[row] : nullptr;
      emit_tails<F, T>(z_lo, 0u, thr, thr_hi, any, s, jg, N, tails, counter, cap, prow, rootS, t);
      emit_tails<F, T>(z_hi, uint32_t(H), thr, thr_hi, any, s, jg, N, tails, counter, cap, prow, rootS, t);
    }
  }
}

// ------------------------------------------------------------ detector pairs --
// The two time-aligned channels a and b of a detector pair (H1 and L1) are
// correlated with one template through one complex inverse transform: the
// paper's packing of a pair into the real and imaginary parts of one complex
// series (Sec. 3.2 step (i)).  With the half spectra (k = 0..M, M = N/2)
//   C^a_k = conj(W_k) A_k,  C^b_k = conj(W_k) B_k      (C_0, C_M real),
// the spectrum of z = N (rho^a + i rho^b) is Q_k = P_k = C^a_k + i C^b_k for
// k <= M and Q_{N-k} = R_k = conj(C^a_k) + i conj(C^b_k).  Its length-N
// inverse transform does not fit one workgroup's registers at N = 2^16, so it
// is split by decimation in frequency over the output parity e:
//   z_{2m+e} = sum_{k<M} A^e_k exp(2 pi i k m / M),
//   A^e_k = (P_k + (-1)^e R_{M-k}) exp(2 pi i k e / N),
// one workgroup per parity, each a length-M transform with the passes of a
// single correlation.  Both workgroups of a (pair, template) read the same
// spectra; they run back to back on one XCD, so the second reads from L2.
//
// pair_pre forms A^e in registers, one register pair (k2, R1-1-k2) at a time:
// under MAP_MIRROR the bins M - k of a thread's two registers are held by
// lane l ^ 32 at the other register of the pair, so the R values cross with
// two lane swaps per register.  Column S1/2 (lane 32 of wave 0) pairs within
// its own register pair.  Column 0 (lane 0 of wave 0) pairs bin S1 k2 with
// S1 (R1 - k2), another register pair: that thread first forms P_k alone
// (plus the Nyquist term at k = 0), keeps its R values in `stash`, and adds
// the partner terms after the loop.
template <class F, int G, int E, typename T, typename TW>
__device__ __forceinline__ void pair_pre(cx<T>* v, double& acc_a, double& acc_b, const uint32_t* cols,
                                         const rsrc_t& rW, const rsrc_t& rA, const rsrc_t& rB,
                                         const cx<T>* __restrict__ tw_u, int t, cx<T>* stash) {
  constexpr int NP = F::R1 / 2;       // register pairs per column
  // register pairs per load group: three spectra per bin load ahead here, so
  // more than two pairs in flight spill
  constexpr int GP = G >= 4 ? 2 : 1;
  static_assert(NP % GP == 0 && F::R1 % 2 == 0, "pair group size");
  constexpr int NG = NP / GP;
  constexpr uint32_t SW = sizeof(TW), SY = sizeof(cx<T>);
  const int lane = t & 63;
  const bool wave0 = __builtin_amdgcn_readfirstlane(t) < 64;
#pragma unroll
  for (int c = 0; c < F::C1; ++c) {
    const uint32_t col = cols[c];
    const bool dc = (c == 0) && (col == 0u);
    cx<T> bu = {T(1), T(0)};
    if constexpr (E == 1) bu = tw_u[col];  // exp(2 pi i col / N)
    TW lw[2][GP][2];
    cx<T> la[2][GP][2], lb[2][GP][2];
    auto issue = [&](int g, int buf) {
#pragma unroll
      for (int p = 0; p < GP; ++p) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = g * GP + p;
          const uint32_t k2 = uint32_t(h ? F::R1 - 1 - i : i);
          lw[buf][p][h] = buf_load<TW>(rW, col * SW, uint32_t(F::S1) * k2 * SW);
          la[buf][p][h] = buf_load<cx<T>>(rA, col * SY, uint32_t(F::S1) * k2 * SY);
          lb[buf][p][h] = buf_load<cx<T>>(rB, col * SY, uint32_t(F::S1) * k2 * SY);
        }
      }
    };
    issue(0, 0);
    static_for<NG>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      if constexpr (g + 1 < NG) issue(g + 1, (g + 1) & 1);
      static_for<GP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int i = g * GP + p;
        constexpr int r1 = i, r2 = F::R1 - 1 - i;
        cx<T> P[2], R[2];
        cx<T> RM = {T(0), T(0)};  // R_M (the Nyquist term) of column 0
        static_for<2>([&](auto hc) {
          constexpr int h = decltype(hc)::value;
          cx<T> wk = load_spec<TW, T>(&lw[g & 1][p][h], 0), ak = la[g & 1][p][h], bk = lb[g & 1][p][h];
          T cma = T(0), cmb = T(0);
          if constexpr (r1 == 0 && h == 0) {
            // slot 0 of column 0 packs the real X_0 (.x) and X_M (.y)
            cma = dc ? wk.y * ak.y : T(0);
            cmb = dc ? wk.y * bk.y : T(0);
            wk.y = dc ? T(0) : wk.y;
            ak.y = dc ? T(0) : ak.y;
            bk.y = dc ? T(0) : bk.y;
          }
          const cx<T> ca = cmulc(wk, ak), cb = cmulc(wk, bk);
          double pa = 2.0 * (double(ca.x) * double(ca.x) + double(ca.y) * double(ca.y));
          double pb = 2.0 * (double(cb.x) * double(cb.x) + double(cb.y) * double(cb.y));
          if constexpr (r1 == 0 && h == 0) {
            pa = dc ? double(ca.x) * double(ca.x) + double(cma) * double(cma) : pa;
            pb = dc ? double(cb.x) * double(cb.x) + double(cmb) * double(cmb) : pb;
            RM = {cma, cmb};
          }
          acc_a += pa;
          acc_b += pb;
          P[h] = {ca.x - cb.y, ca.y + cb.x};
          R[h] = {ca.x + cb.y, cb.x - ca.y};
        });
        cx<T> X0, X1;  // R_{M-k} for the bins of registers r1 and r2
        partner_pair(R[0], R[1], X0, X1);
        if (c == 0 && wave0) {
          if (lane == 32) {  // column S1/2: its partners are its own two registers
            X0 = R[1];
            X1 = R[0];
          }
          if (lane == 0) {  // column 0: the partner terms are added after the loop
            X0 = r1 == 0 ? RM : cx<T>{T(0), T(0)};
            X1 = cx<T>{T(0), T(0)};
            stash[r1] = R[0];
            stash[r2] = R[1];
          }
        }
        if constexpr (E == 0) {
          v[c * F::R1 + r1] = cadd(P[0], X0);
          v[c * F::R1 + r2] = cadd(P[1], X1);
        } else {
          v[c * F::R1 + r1] = cmul(rot<r1, 2 * F::R1, +1>(bu), csub(P[0], X0));
          v[c * F::R1 + r2] = cmul(rot<r2, 2 * F::R1, +1>(bu), csub(P[1], X1));
        }
        pin(v[c * F::R1 + r1]);
        pin(v[c * F::R1 + r2]);
      });
      pin(acc_a);
      pin(acc_b);
      sched_fence();
    });
    if (c == 0 && wave0 && lane == 0) {
      // column 0: bin S1 r pairs with bin S1 (R1 - r); exp(2 pi i S1 r / N) = exp(i pi r / R1)
      static_for<F::R1 - 1>([&](auto rc) {
        constexpr int r = decltype(rc)::value + 1;
        const cx<T> x = stash[F::R1 - r];
        if constexpr (E == 0)
          v[r] = cadd(v[r], x);
        else
          v[r] = csub(v[r], rot<r, 2 * F::R1, +1>(x));
      });
    }
    sched_fence();
  }
}

// Stage 3 of a pair workgroup of parity E, threshold: register i holds
// z = N (rho^a + i rho^b) at lag 2 n + E (n the output index).  Component x
// is channel a (segment sa, threshold thr[0]), y is channel b.
template <class F, int E, typename T>
__device__ __forceinline__ void emit_pair_tails(const cx<T>* v, const T* thr, const T* thr_hi, bool any,
                                                const uint32_t* seg, uint32_t j, double N,
                                                tail_rec_t<T>* __restrict__ tails, unsigned long long* __restrict__ counter,
                                                uint64_t cap, unsigned long long* const* prow, const double* rootS,
                                                int t) {
  const int lane = t & 63;
  auto is_tail = [&](T val, int h) { return any && (fabs(val) > thr[h]) && (fabs(val) < thr_hi[h]); };
  uint32_t cnt = 0;
#pragma unroll
  for (int i = 0; i < F::P; ++i) cnt += uint32_t(is_tail(v[i].x, 0)) + uint32_t(is_tail(v[i].y, 1));
  uint32_t incl = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(incl, d, 64);
    if (lane >= d) incl += o;
  }
  const uint32_t total = __shfl(incl, 63, 64);
  if (total == 0) return;
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(counter, (unsigned long long)total);
  base = __shfl(base, 0, 64);
  if (cnt == 0) return;
  uint64_t idx = base + (incl - cnt);
#pragma unroll
  for (int c = 0; c < F::C2; ++c) {
#pragma unroll
    for (int mp = 0; mp < F::R3; ++mp) {
      const uint32_t lag = 2u * uint32_t(fft3_out_index<F>(t, c, mp)) + uint32_t(E);
      const cx<T> a = v[c * F::R3 + mp];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        T val = h ? a.y : a.x;
        asm volatile("" : "+v"(val));
        if (!is_tail(val, h)) continue;
        if (prow[h]) {
          const float snr = float(fabs(double(val)) / rootS[h]);
          const unsigned long long key = (static_cast<unsigned long long>(__float_as_uint(snr)) << 32) |
                                         (static_cast<unsigned long long>(0x7fffffffu - j) << 1) |
                                         (val < T(0) ? 1ull : 0ull);
          atomicMax(prow[h] + lag, key);
        } else if (idx < cap) {
          tail_rec_t<T> r{};
          r.segment = seg[h];
          r.template_id = j;
          r.lag = lag;
          r.rho = decltype(r.rho)(double(val) / N);
          tails[idx] = r;
        }
        ++idx;
      }
    }
  }
}

template <typename T, typename TW, class F, bool DENSE, int G, int E>
__device__ __forceinline__ void pair_body(T* lds, double* red, cx<T>* stash, const rsrc_t& rW, const rsrc_t& rA,
                                          const rsrc_t& rB, const uint32_t* seg, const uint32_t* prow_row, uint32_t jg,
                                          const cx<T>* __restrict__ tw_u, const cx<T>* __restrict__ tw1,
                                          const cx<T>* tw2, double kappa, double kappa_hi,
                                          double* __restrict__ sigma_out, uint32_t k_total, tail_rec_t<T>* __restrict__ tails,
                                          unsigned long long* __restrict__ counter, uint64_t cap,
                                          unsigned long long* __restrict__ proj, const uint64_t* __restrict__ proj_off,
                                          T* __restrict__ rho_dense, int t) {
  constexpr int M = F::M;
  constexpr double N = 2.0 * M;
  cx<T> v[F::P];
  double acc_a = 0.0, acc_b = 0.0;
  uint32_t cols[F::C1];
#pragma unroll
  for (int c = 0; c < F::C1; ++c) cols[c] = fft3_col<F, MAP_MIRROR>(t, c);
  pair_pre<F, G, E, T, TW>(v, acc_a, acc_b, cols, rW, rA, rB, tw_u, t, stash);
  double Sb = 0.0;
  const double Sa = corr_ifft<F, T, 2, false, tw2_in_lds<F>()>(v, lds, red, cols, tw1, tw2, t, acc_a, acc_b, &Sb);
  const double rootS[2] = {sqrt(Sa), sqrt(Sb)};
  if (E == 0 && t == 0 && sigma_out) {
    sigma_out[uint64_t(seg[0]) * k_total + jg] = rootS[0] / N;
    sigma_out[uint64_t(seg[1]) * k_total + jg] = rootS[1] / N;
  }
  if constexpr (DENSE) {
    const T inv = T(1.0 / N);
    T* ra = rho_dense + (uint64_t(seg[0]) * k_total + jg) * uint64_t(2 * M);
    T* rb = rho_dense + (uint64_t(seg[1]) * k_total + jg) * uint64_t(2 * M);
#pragma unroll
    for (int c = 0; c < F::C2; ++c) {
#pragma unroll
      for (int mp = 0; mp < F::R3; ++mp) {
        const uint32_t lag = 2u * uint32_t(fft3_out_index<F>(t, c, mp)) + uint32_t(E);
        ra[lag] = v[c * F::R3 + mp].x * inv;
        rb[lag] = v[c * F::R3 + mp].y * inv;
      }
    }
  } else {
    const T thr[2] = {T(kappa * rootS[0]), T(kappa * rootS[1])};
    const T thr_hi[2] = {kappa_hi > 0.0 ? T(kappa_hi * rootS[0]) : T(INFINITY),
                         kappa_hi > 0.0 ? T(kappa_hi * rootS[1]) : T(INFINITY)};
    T ma = T(0), mb = T(0);
#pragma unroll
    for (int i = 0; i < F::P; ++i) {
      ma = fmax(ma, fabs(v[i].x));
      mb = fmax(mb, fabs(v[i].y));
    }
    const bool any = (ma > thr[0] && rootS[0] > 0.0) || (mb > thr[1] && rootS[1] > 0.0);
    if (__ballot(any)) {
      unsigned long long* prow[2] = {proj ? proj + proj_off[prow_row[0]] : nullptr,
                                     proj ? proj + proj_off[prow_row[1]] : nullptr};
      emit_pair_tails<F, E, T>(v, thr, thr_hi, any, seg, jg, N, tails, counter, cap, prow, rootS, t);
    }
  }
}

// One workgroup per (template j, pair row r) in the order of tile_map over n_rows = 2 x pairs
// rows: pair q = r / 2, parity e = r % 2; its channels are spectrum rows 2q (a) and 2q + 1 (b)
// of yspec, with the segment ids seg_ids[2q], seg_ids[2q + 1] (or row0 + those rows).  Other
// arguments as corr_kernel.
template <typename T, typename TW, class F, bool DENSE, int G>
__global__ __launch_bounds__(F::NT) void pair_kernel(
    const TW* __restrict__ bank, const cx<T>* __restrict__ yspec, const uint32_t* __restrict__ seg_ids,
    const cx<T>* __restrict__ tw_u, const cx<T>* __restrict__ tw1, const cx<T>* __restrict__ tw2,
    uint32_t K, uint32_t n_rows, uint32_t tile, double kappa, double* __restrict__ sigma_out,
    tail_rec_t<T>* __restrict__ tails, unsigned long long* __restrict__ counter, uint64_t cap,
    unsigned long long* __restrict__ proj, const uint64_t* __restrict__ proj_off, double kappa_hi,
    T* __restrict__ rho_dense, uint32_t j0, uint32_t k_total, uint32_t row0) {
  constexpr int M = F::M;
  __shared__ T lds[F::LDS_ELEMS];
  __shared__ double red[2 * F::NW];
  __shared__ cx<T> stash[F::R1];
  constexpr bool TWL = tw2_in_lds<F>();
  __shared__ cx<T> tw2s[TWL ? F::R2 * F::R3 : 1];
  const int t = threadIdx.x;
  uint32_t j, row;
  if (!tile_map(blockIdx.x, K, n_rows, tile, j, row)) return;
  if constexpr (TWL) fft3_tw2_stage<F>(tw2s, tw2, t);
  const uint32_t ra = row & ~1u, rb = ra + 1u;
  const uint32_t seg[2] = {uint32_t(__builtin_amdgcn_readfirstlane(seg_ids ? seg_ids[ra] : row0 + ra)),
                           uint32_t(__builtin_amdgcn_readfirstlane(seg_ids ? seg_ids[rb] : row0 + rb))};
  const uint32_t prow_row[2] = {ra, rb};
  const uint32_t jg = j0 + j;
  const rsrc_t rW = make_rsrc(bank + uint64_t(j) * M, uint32_t(M) * uint32_t(sizeof(TW)));
  const rsrc_t rA = make_rsrc(yspec + uint64_t(ra) * M, uint32_t(M) * uint32_t(sizeof(cx<T>)));
  const rsrc_t rB = make_rsrc(yspec + uint64_t(rb) * M, uint32_t(M) * uint32_t(sizeof(cx<T>)));
  if (row & 1u)
    pair_body<T, TW, F, DENSE, G, 1>(lds, red, stash, rW, rA, rB, seg, prow_row, jg, tw_u, tw1, TWL ? tw2s : tw2, kappa,
                                     kappa_hi, sigma_out, k_total, tails, counter, cap, proj, proj_off, rho_dense, t);
  else
    pair_body<T, TW, F, DENSE, G, 0>(lds, red, stash, rW, rA, rB, seg, prow_row, jg, tw_u, tw1, TWL ? tw2s : tw2, kappa,
                                     kappa_hi, sigma_out, k_total, tails, counter, cap, proj, proj_off, rho_dense, t);
}

}  // namespace bfs
