// Kernels of the runtime that are not templates (one definition, in the
// library's runtime source): filling counters, compacting projection keys,
// finding coincidences of detector pairs, the unit-norm factors of fused
// synthesis.
#pragma once

#include "bfs_kernels.h"

namespace bfs {

__global__ void fill_u64_kernel(unsigned long long* p, uint64_t n, unsigned long long v) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Projection keys -> list of (index, key) for every nonzero key (order
// arbitrary; the host sorts), one atomicAdd per wave.  Entries past cap are
// counted but not written.
__global__ __launch_bounds__(256) void project_compact_kernel(const unsigned long long* __restrict__ keys, uint64_t n,
                                                              unsigned long long* __restrict__ list,
                                                              unsigned long long* __restrict__ counter, uint64_t cap) {
  const int lane = threadIdx.x & 63;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t base_i = uint64_t(blockIdx.x) * blockDim.x; base_i < n; base_i += stride) {
    const uint64_t i = base_i + threadIdx.x;
    const unsigned long long key = i < n ? keys[i] : 0ull;
    const bool pred = key != 0ull;
    const uint64_t mask = __ballot(pred);
    if (!mask) continue;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader, 64);
    if (pred) {
      const uint64_t idx = base + __popcll(mask & below);
      if (idx < cap) {
        list[2 * idx] = i;
        list[2 * idx + 1] = key;
      }
    }
  }
}

// Coincidences of detector pairs (Sec. 5, Table 3).  Pair p's channels are
// caller segments 2p and 2p + 1, their projection keys at proj + lag0[2p] and
// proj + lag0[2p + 1] (N_p = lag0[2p + 1] - lag0[2p] lags each).  A lag where
// both keys are set and the winning templates' initial frequencies differ by
// less than delta (FP64) becomes {pair, lag, template_a, template_b, snr_a,
// snr_b}, one atomicAdd per wave; records past cap are counted, not written.
struct coinc_rec {
  uint32_t pair, lag, template_a, template_b;
  float snr_a, snr_b;
};

__device__ __forceinline__ void decode_key(unsigned long long key, uint32_t& j, float& snr) {
  const uint32_t lo = uint32_t(key & 0xffffffffull);
  j = 0x7fffffffu - (lo >> 1);
  snr = __uint_as_float(uint32_t(key >> 32));
  if (lo & 1u) snr = -snr;
}

__global__ __launch_bounds__(256) void coinc_kernel(const unsigned long long* __restrict__ proj,
                                                    const uint64_t* __restrict__ lag0, const double* __restrict__ f0,
                                                    double delta, coinc_rec* __restrict__ out,
                                                    unsigned long long* __restrict__ counter, uint64_t cap) {
  const uint32_t p = blockIdx.y;
  const uint64_t base = lag0[2 * p];
  const uint64_t np = lag0[2 * p + 1] - base;
  const uint64_t n = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  bool pred = false;
  uint32_t ja = 0, jb = 0;
  float sa = 0.f, sb = 0.f;
  if (n < np) {
    const unsigned long long ka = proj[base + n], kb = proj[base + np + n];
    if (ka && kb) {
      decode_key(ka, ja, sa);
      decode_key(kb, jb, sb);
      pred = fabs(f0[ja] - f0[jb]) < delta;
    }
  }
  const uint64_t mask = __ballot(pred);
  if (!mask) return;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned long long b0 = 0;
  if (lane == leader) b0 = atomicAdd(counter, (unsigned long long)__popcll(mask));
  b0 = __shfl(b0, leader, 64);
  if (!pred) return;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint64_t idx = b0 + __popcll(mask & below);
  if (idx < cap) out[idx] = coinc_rec{p, uint32_t(n), ja, jb, sa, sb};
}

// A finished job's counters and the head of each result list, copied into
// pinned host memory by the job's own stream right after its kernels, while
// the CUs are free.  (A copy queued from the host later runs as a blit kernel
// and, once the next job's persistent correlation kernel holds every CU,
// waits for that whole kernel.)  counter[0..2] counts tails, projection
// entries and coincidences; list i gets min(counter[i], cap) entries of
// `words` 8-byte words (dst null: nothing).
struct PublishList {
  const uint2* src;
  uint2* dst;
  uint64_t cap;
  uint32_t words;
};

__global__ __launch_bounds__(256) void publish_kernel(const unsigned long long* __restrict__ counter,
                                                      unsigned long long* __restrict__ count_dst, PublishList l0,
                                                      PublishList l1, PublishList l2) {
  if (blockIdx.x == 0 && threadIdx.x < 3) count_dst[threadIdx.x] = counter[threadIdx.x];
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  const uint64_t t0 = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  auto copy = [&](const PublishList& l, unsigned long long cnt) {
    if (!l.dst) return;
    const uint64_t n = (uint64_t(cnt) < l.cap ? uint64_t(cnt) : l.cap) * l.words;
    for (uint64_t i = t0; i < n; i += stride) l.dst[i] = l.src[i];
  };
  copy(l0, counter[0]);
  copy(l1, counter[1]);
  copy(l2, counter[2]);
}

// FP64 energy sum_m w[m]^2 of each grid chirp (the unit-norm factor of the
// fused kernel is 1 / sqrt of it, as the resident bank's unpack applies).
// One workgroup per template; the samples are the chirp_sample values.
__global__ __launch_bounds__(256) void chirp_norm_kernel(const double* __restrict__ f0, const double* __restrict__ fdot,
                                                         const uint32_t* __restrict__ len, double fs, int taper,
                                                         int sym, float* __restrict__ norm) {
  __shared__ double red[4];
  const uint32_t j = blockIdx.x;
  const int L = int(len[j]);
  double acc = 0.0;
  for (int m = threadIdx.x; m < L; m += 256) {
    double a = chirp_sample(m, L, f0[j], fdot[j], fs, taper);
    if (sym) a += chirp_sample(L - 1 - m, L, f0[j], fdot[j], fs, taper);
    acc += a * a;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double e = red[0] + red[1] + red[2] + red[3];
    norm[j] = e > 0.0 ? float(1.0 / sqrt(e)) : 0.0f;
  }
}

}  // namespace bfs
