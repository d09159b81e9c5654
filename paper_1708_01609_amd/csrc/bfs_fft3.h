// Register-resident three-pass FFT of length M = R1*R2*R3 for one workgroup
// of NT threads.  Every thread keeps P = M/NT complex points in registers.
//
// Index map (decimation in time, sign DIR):
//   input  k = col + S1*k2            (S1 = R2*R3, col = j1 + R3*j2)
//   output n = n0 + R1*m0 + R1*R2*m'
//   pass 1: per column col, DFT_R1 over k2 -> n0, twiddle w_M^(n0*col)
//   pass 2: per item (n0, j1), DFT_R2 over j2 -> m0, twiddle w_S1^(m0*j1)
//   pass 3: per item (n0, m0), DFT_R3 over j1 -> m'
// Thread t owns pass-1 columns t + NT*c (c < P/R1), pass-2 items t + NT*c
// with n0 = item / R3, j1 = item % R3, and pass-3 items t + NT*c with
// n0 = item / R2, m0 = item % R2.  With R2 == R3 the R3 threads that share
// an n0 are consecutive lanes of one wave, so the pass-2 -> pass-3 exchange
// stays inside the wave and needs no workgroup barrier.  The pass-1 ->
// pass-2 exchange spans the workgroup.  Both exchanges go through LDS one
// real plane at a time (x, then y), which halves the LDS footprint: for
// M = 32768 FP32 a plane is 128 KiB of the 160 KiB a CU has.
#pragma once

#include "bfs_device.h"

namespace bfs {

template <typename T, int R1_, int R2_, int R3_, int NT_>
struct Fft3 {
  using real = T;
  static constexpr int R1 = R1_, R2 = R2_, R3 = R3_, NT = NT_;
  static constexpr int M = R1 * R2 * R3;
  static constexpr int P = M / NT;
  static constexpr int S1 = R2 * R3;
  static constexpr int C1 = P / R1;  // pass-1 columns per thread
  static constexpr int C2 = P / R2;  // pass-2 (and pass-3) items per thread
  static constexpr int NW = NT / 64;
  // exchange 1: R1 rows of S1 columns, rows padded so that the R3-lane groups
  // of one wave fall on disjoint LDS banks
  static constexpr int EX1_ROW = S1 + R3;
  static constexpr int EX1_ELEMS = R1 * EX1_ROW;
  // exchange 2: per wave, (64/R3)*C2 groups of R2 rows of R3 (+1 pad) values
  static constexpr int EX2_ROW = R3 + 1;
  static constexpr int EX2_WAVE = (64 / R3) * C2 * R2 * EX2_ROW;
  static constexpr int EX2_ELEMS = NW * EX2_WAVE;
  static constexpr int LDS_ELEMS = EX1_ELEMS > EX2_ELEMS ? EX1_ELEMS : EX2_ELEMS;

  static_assert(R2 == R3, "pass-2/pass-3 exchange is wave-local only for R2 == R3");
  static_assert(NT % 64 == 0, "whole waves only");
  static_assert(64 % R3 == 0, "an n0 group must sit inside one wave");
  static_assert(C1 * R1 == P && C2 * R2 == P, "points per thread must be a multiple of every radix");
  static_assert(S1 == NT * C1, "columns must tile the threads");
};

// LDS fences.  A workgroup barrier orders LDS traffic across waves; inside a
// wave the LDS executes a wave's instructions in order, so a compiler-level
// fence is enough between a wave's own writes and reads.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroup barrier for LDS traffic only: every wave's LDS accesses have
// completed before any wave passes it, and the compiler moves no memory
// access across it.  Unlike __syncthreads it does not wait for the wave's
// outstanding global stores (its release fence would), so stores issued
// before it keep draining while the workgroup goes on.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Phase boundary: no instruction and no memory access moves across it, which
// bounds how many loads the compiler keeps in flight (and registers live).
__device__ __forceinline__ void sched_fence() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// Pin a value in registers at this point: the empty asm "uses and redefines"
// it, so its computation cannot sink past later phase boundaries (which would
// keep that computation's inputs live and spill).
template <typename T>
__device__ __forceinline__ void pin(cx<T>& a) {
  asm volatile("" : "+v"(a.x), "+v"(a.y));
}
__device__ __forceinline__ void pin(double& a) { asm volatile("" : "+v"(a)); }

// Pass-1 column of slot c of thread t.
//  MAP_PLAIN        column = t + NT c.
//  MAP_MIRROR       a column and its Hermitian partner S1 - col sit in lanes
//                   l and l ^ 32 of one wave (lane 32 of the first wave takes
//                   the self-paired column S1/2; column 0 pairs with itself).
//  MAP_MIRROR_ODD   partners col and S1 - 1 - col in lanes l and l ^ 32 (the
//                   pairing of the odd half of a split transform; no column
//                   pairs with itself).
enum ColMap : int { MAP_PLAIN = 0, MAP_MIRROR = 1, MAP_MIRROR_ODD = 2 };

template <class F, int MAP>
__device__ __forceinline__ uint32_t fft3_col(int t, int c) {
  const uint32_t tv = uint32_t(t + F::NT * c);
  if constexpr (MAP == MAP_PLAIN) {
    return tv;
  } else {
    const uint32_t w = tv >> 6, l = tv & 63u;
    const uint32_t lo = 32u * w + l;
    uint32_t hi;
    if constexpr (MAP == MAP_MIRROR)
      hi = (tv == 32u) ? uint32_t(F::S1 / 2) : uint32_t(F::S1) - 32u * w - (l - 32u);
    else
      hi = uint32_t(F::S1 - 1) - 32u * w - (l - 32u);
    return l < 32u ? lo : hi;
  }
}

// v[i] *= w^i for i = 1..R-1, w = exp(DIR 2 pi i e / D) for a per-thread e.
// tab is a [R][stride] table of exp(+2 pi i r e / D) (row r, column e).  The
// thread loads row 1 and every eighth row (anchors) and walks a running
// power w^i = w^(i-1) w between anchors, so each twiddle is at most seven
// products from an exact table value and only a handful of registers stay
// live.  The anchors are requested (twiddle_load) ahead of the arithmetic
// that precedes their use, so the wait for them finds them arrived.
template <int R, typename T>
struct Anchors {
  static constexpr int NA = R > 1 ? 1 + (R - 1) / 8 : 1;  // row 1, rows 8, 16, ...
  cx<T> a[NA];
};

template <int R, typename T>
__device__ __forceinline__ Anchors<R, T> twiddle_load(const cx<T>* __restrict__ tab, uint32_t stride, uint32_t e) {
  Anchors<R, T> w{};
  if constexpr (R > 1) {
    const rsrc_t rt = make_rsrc(tab, uint32_t(R) * stride * uint32_t(sizeof(cx<T>)));
    const uint32_t voff = e * uint32_t(sizeof(cx<T>));
    w.a[0] = buf_load<cx<T>>(rt, voff, stride * uint32_t(sizeof(cx<T>)));
#pragma unroll
    for (int k = 1; k < Anchors<R, T>::NA; ++k)
      w.a[k] = buf_load<cx<T>>(rt, voff, uint32_t(8 * k) * stride * uint32_t(sizeof(cx<T>)));
  }
  return w;
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void twiddle_apply(cx<T>* v, const Anchors<R, T>& an) {
  if constexpr (R > 1) {
    cx<T> w1 = an.a[0];
    if constexpr (DIR < 0) w1.y = -w1.y;
    cx<T> w = w1;
#pragma unroll
    for (int i = 1; i < R; ++i) {
      if (i % 8 == 0) {
        w = an.a[i / 8];
        if constexpr (DIR < 0) w.y = -w.y;
      } else if (i > 1) {
        w = cmul(w, w1);
      }
      v[i] = cmul(v[i], w);
    }
  }
}

// Pass 1: DFT over k2 for every owned column, then the w_M^(n0*col) twiddle
// (tw1 holds exp(+2 pi i n0 col / M) as [n0][col]; DIR < 0 uses its conjugate).
template <class F, int DIR, typename T>
__device__ __forceinline__ void fft3_pass1(cx<T>* v, const cx<T>* __restrict__ tw1, const uint32_t* cols) {
#pragma unroll
  for (int c = 0; c < F::C1; ++c) {
    const Anchors<F::R1, T> an = twiddle_load<F::R1, T>(tw1, F::S1, cols[c]);
    dft<F::R1, DIR, T>(&v[c * F::R1]);
    twiddle_apply<F::R1, DIR, T>(&v[c * F::R1], an);
    sched_fence();
  }
}

// Exchange 1 for one plane (PL = 0: x, 1: y): write pass-1 outputs, barrier,
// read pass-2 inputs.  The caller places the barrier between planes.
template <class F, int PL, typename T>
__device__ __forceinline__ void fft3_ex1_write(const cx<T>* v, T* lds, const uint32_t* cols) {
  // rows go in blocks of 16 from one base address each, so every offset fits
  // the 16-bit immediate of ds_write and no per-row address stays live
  constexpr int RB = 16;
#pragma unroll
  for (int c = 0; c < F::C1; ++c) {
#pragma unroll
    for (int blk = 0; blk * RB < F::R1; ++blk) {
      uint32_t boff = uint32_t(blk * RB * F::EX1_ROW);
      asm volatile("" : "+s"(boff));  // keep the block base opaque: one add, then immediates
      T* pb = lds + boff + cols[c];
#pragma unroll
      for (int r = 0; r < RB && blk * RB + r < F::R1; ++r) {
        const cx<T> a = v[c * F::R1 + blk * RB + r];
        pb[r * F::EX1_ROW] = PL == 0 ? a.x : a.y;
      }
    }
  }
}
template <class F, int PL, typename T>
__device__ __forceinline__ void fft3_ex1_read(cx<T>* v, const T* lds, int t) {
#pragma unroll
  for (int c = 0; c < F::C2; ++c) {
    const int item = t + F::NT * c;
    const int n0 = item / F::R3, j1 = item % F::R3;
#pragma unroll
    for (int j2 = 0; j2 < F::R2; ++j2) {
      const T a = lds[n0 * F::EX1_ROW + j1 + F::R3 * j2];
      if constexpr (PL == 0) v[c * F::R2 + j2].x = a;
      else v[c * F::R2 + j2].y = a;
    }
  }
}

// Pass 2: DFT over j2 for every owned item, then w_S1^(m0*j1) (tw2 is
// exp(+2 pi i m0 j1 / S1) as [m0][j1]).  fft3_pass2_load requests the
// anchors; callers issue it before exchange 1, whose barriers hide the wait.
template <class F, typename T>
struct Pass2Anchors {
  Anchors<F::R2, T> an[F::C2];
};
template <class F, typename T>
__device__ __forceinline__ Pass2Anchors<F, T> fft3_pass2_load(const cx<T>* __restrict__ tw2, int t) {
  Pass2Anchors<F, T> p;
#pragma unroll
  for (int c = 0; c < F::C2; ++c) p.an[c] = twiddle_load<F::R2, T>(tw2, F::R3, uint32_t(t + F::NT * c) % F::R3);
  return p;
}
template <class F, int DIR, typename T>
__device__ __forceinline__ void fft3_pass2(cx<T>* v, const Pass2Anchors<F, T>& p) {
#pragma unroll
  for (int c = 0; c < F::C2; ++c) {
    dft<F::R2, DIR, T>(&v[c * F::R2]);
    sched_fence();
    twiddle_apply<F::R2, DIR, T>(&v[c * F::R2], p.an[c]);
    sched_fence();
  }
}
template <class F, int DIR, typename T>
__device__ __forceinline__ void fft3_pass2(cx<T>* v, const cx<T>* __restrict__ tw2, int t) {
  fft3_pass2<F, DIR, T>(v, fft3_pass2_load<F, T>(tw2, t));
}

// v[i] *= tab[i stride + e] for i = 1..R-1 (conjugated for DIR < 0), with tab
// an LDS table: every twiddle is read (one ds_read each, offsets as
// immediates from one base register), none is formed by products.
template <int R, int DIR, typename T>
__device__ __forceinline__ void twiddle_apply_lds(cx<T>* v, const cx<T>* tab, uint32_t stride, uint32_t e) {
  // the column's LDS byte address, opaque: one register, and each row's read
  // takes its offset as an immediate (the table may lie beyond the 16-bit
  // offset range from LDS address 0)
  using lcx = __attribute__((address_space(3))) const cx<T>;
  uint32_t a = uint32_t(uintptr_t((lcx*)(tab + e)));
  asm volatile("" : "+v"(a));
  lcx* col = (lcx*)(uintptr_t(a));
#pragma unroll
  for (int i = 1; i < R; ++i) {
    cx<T> w = {col[i * stride].x, col[i * stride].y};
    if constexpr (DIR < 0) w.y = -w.y;
    v[i] = cmul(v[i], w);
  }
}

// Pass 2 with the twiddle table tw2 ([R2][R3], exp(+2 pi i m0 j1 / S1)) held in
// LDS.  fft3_tw2_stage copies the table; a workgroup barrier of the caller
// (exchange 1) orders the copy before the reads.  Used by the 1024-thread
// shapes (32 points per thread, one inverse transform per workgroup), where it
// measured faster; smaller workgroups pay the per-correlation copy for fewer
// products saved, and the split kernel's two transforms measured slower.
template <class F>
constexpr bool tw2_in_lds() {
  return F::NT == 1024;
}
template <class F, typename T>
__device__ __forceinline__ void fft3_tw2_stage(cx<T>* tw2s, const cx<T>* __restrict__ tw2, int t) {
  for (int i = t; i < F::R2 * F::R3; i += F::NT) tw2s[i] = tw2[i];
}
template <class F, int DIR, typename T>
__device__ __forceinline__ void fft3_pass2_tab(cx<T>* v, const cx<T>* tw2s, int t) {
#pragma unroll
  for (int c = 0; c < F::C2; ++c) {
    dft<F::R2, DIR, T>(&v[c * F::R2]);
    sched_fence();
    twiddle_apply_lds<F::R2, DIR, T>(&v[c * F::R2], tw2s, F::R3, uint32_t(t + F::NT * c) % F::R3);
    sched_fence();
  }
}

template <class F, typename T>
__device__ __forceinline__ void fft3_ex2(cx<T>* v, T* lds, int t) {
  const int lane = t & 63, wave = t >> 6;
  T* base = lds + wave * F::EX2_WAVE;
  const int g = lane / F::R3, q = lane % F::R3;
#pragma unroll
  for (int pl = 0; pl < 2; ++pl) {
#pragma unroll
    for (int c = 0; c < F::C2; ++c) {
      T* grp = base + (c * (64 / F::R3) + g) * F::R2 * F::EX2_ROW;
#pragma unroll
      for (int m0 = 0; m0 < F::R2; ++m0) grp[m0 * F::EX2_ROW + q] = pl == 0 ? v[c * F::R2 + m0].x : v[c * F::R2 + m0].y;
    }
    wave_lds_fence();
#pragma unroll
    for (int c = 0; c < F::C2; ++c) {
      const T* grp = base + (c * (64 / F::R3) + g) * F::R2 * F::EX2_ROW;
#pragma unroll
      for (int j1 = 0; j1 < F::R3; ++j1) {
        const T a = grp[q * F::EX2_ROW + j1];
        if (pl == 0) v[c * F::R3 + j1].x = a;
        else v[c * F::R3 + j1].y = a;
      }
    }
    wave_lds_fence();
  }
}

template <class F, int DIR, typename T>
__device__ __forceinline__ void fft3_pass3(cx<T>* v) {
#pragma unroll
  for (int c = 0; c < F::C2; ++c) dft<F::R3, DIR, T>(&v[c * F::R3]);
}

// Output index of register slot (c, m') after pass 3 for thread t.
template <class F>
__device__ __forceinline__ int fft3_out_index(int t, int c, int mp) {
  const int item = t + F::NT * c;
  const int n0 = item / F::R2, m0 = item % F::R2;
  return n0 + F::R1 * m0 + F::R1 * F::R2 * mp;
}

}  // namespace bfs
