// Device building blocks for the gfx950 matched-filter kernels: a complex
// type, compile-time twiddle constants, in-register DFTs of radix 2..64,
// wave reductions and the storage formats of template spectra.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace bfs {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.x, -a.y}; }

// ------------------------------------------------------------------------
// Compile-time cos/sin of 2*pi*num/den.  The angle is reduced exactly in
// integers to [0, pi/4] and evaluated by Taylor series in double, which
// gives the constants to about one ulp of double.
constexpr double kPiHalf = 1.57079632679489661923132169163975144;

constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int i = 1; i < 16; ++i) {
    term *= -x2 / double((2 * i) * (2 * i + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int i = 1; i < 16; ++i) {
    term *= -x2 / double((2 * i - 1) * (2 * i));
    sum += term;
  }
  return sum;
}
// returns cos (which = 0) or sin (which = 1) of 2*pi*num/den
constexpr double cs2pi(long num, long den, int which) {
  num %= den;
  if (num < 0) num += den;
  const long q = (4 * num) / den;          // quadrant
  long r = 4 * num - q * den;              // angle within quadrant = (pi/2) r / den
  bool swap = false;
  if (2 * r > den) {                        // use the complementary angle
    r = den - r;
    swap = true;
  }
  const double th = kPiHalf * double(r) / double(den);
  double c = taylor_cos(th), s = taylor_sin(th);
  if (swap) {
    const double tmp = c;
    c = s;
    s = tmp;
  }
  // rotate by q quarter turns
  double cc = c, ss = s;
  if (q == 1) { cc = -s; ss = c; }
  if (q == 2) { cc = -c; ss = -s; }
  if (q == 3) { cc = s; ss = -c; }
  return which == 0 ? cc : ss;
}

// ------------------------------------------------------------------------
template <int... Is, typename F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, Is...>, F&& f) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

// a * exp(DIR * 2*pi*i * K / R) with the rotation known at compile time;
// exact for multiples of a quarter turn, 2 mul + 2 add for odd eighths.
template <int K, int R, int DIR, typename T>
__device__ __forceinline__ cx<T> rot(cx<T> a) {
  constexpr long k = ((long(K) % R) + R) % R;
  if constexpr (k == 0) {
    return a;
  } else if constexpr (2 * k == R) {
    return {-a.x, -a.y};
  } else if constexpr (4 * k == R) {           // exp(DIR i pi/2) = DIR i
    if constexpr (DIR > 0) return {-a.y, a.x};
    else return {a.y, -a.x};
  } else if constexpr (4 * k == 3 * R) {       // -DIR i
    if constexpr (DIR > 0) return {a.y, -a.x};
    else return {-a.y, a.x};
  } else if constexpr ((8 * k) % R == 0) {     // odd multiple of pi/4
    constexpr T h = T(0.707106781186547524400844362104849039);
    constexpr int oct = int(8 * k / R);         // 1, 3, 5, 7
    // exp(i s pi/4) with s = DIR*oct: cos = sx*h, sin = sy*h
    constexpr int sx = (oct == 1 || oct == 7) ? 1 : -1;
    constexpr int sy0 = (oct == 1 || oct == 3) ? 1 : -1;
    constexpr int sy = DIR > 0 ? sy0 : -sy0;
    // (a.x + i a.y)(sx + i sy) h
    T re, im;
    if constexpr (sx > 0 && sy > 0) { re = a.x - a.y; im = a.x + a.y; }
    else if constexpr (sx > 0 && sy < 0) { re = a.x + a.y; im = a.y - a.x; }
    else if constexpr (sx < 0 && sy > 0) { re = -a.x - a.y; im = a.x - a.y; }
    else { re = a.y - a.x; im = -a.x - a.y; }
    return {re * h, im * h};
  } else {
    constexpr T c = T(cs2pi(k, R, 0));
    constexpr T s = T(DIR > 0 ? cs2pi(k, R, 1) : -cs2pi(k, R, 1));
    return {a.x * c - a.y * s, a.x * s + a.y * c};
  }
}

template <typename T>
__device__ __forceinline__ T fmad(T a, T b, T c) {
  if constexpr (std::is_same_v<T, float>) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}

// Radix-2 butterfly with a compile-time twiddle, fused-multiply-add form:
//   x0 = e + w o,  x1 = e - w o,  w = exp(DIR 2 pi i K / R).
// Trivial rotations cost 4 additions.  Otherwise the larger of cos and sin
// is factored out (Linzer and Feig's FMA butterfly): with |c| >= |s|,
// w o = c (o.x - t o.y, o.y + t o.x), t = s / c, so the pair costs 6 FMAs
// instead of 4 multiply/FMAs plus 4 additions; odd eighths use 2 additions
// and 4 FMAs with +-1/sqrt(2).
template <int K, int R, int DIR, typename T>
__device__ __forceinline__ void bfly(const cx<T>& e, const cx<T>& o, cx<T>& x0, cx<T>& x1) {
  constexpr long k = ((long(K) % R) + R) % R;
  if constexpr (k == 0 || 2 * k == R || 4 * k == R || 4 * k == 3 * R) {
    const cx<T> t = rot<K, R, DIR>(o);
    x0 = cadd(e, t);
    x1 = csub(e, t);
  } else if constexpr ((8 * k) % R == 0) {
    constexpr T h = T(0.707106781186547524400844362104849039);
    constexpr int oct = int(8 * k / R);
    constexpr int sx = (oct == 1 || oct == 7) ? 1 : -1;
    constexpr int sy0 = (oct == 1 || oct == 3) ? 1 : -1;
    constexpr int sy = DIR > 0 ? sy0 : -sy0;
    // w o = h (sx o.x - sy o.y, sy o.x + sx o.y)
    T ux, uy;
    if constexpr (sx > 0 && sy > 0) { ux = o.x - o.y; uy = o.x + o.y; }
    else if constexpr (sx > 0 && sy < 0) { ux = o.x + o.y; uy = o.y - o.x; }
    else if constexpr (sx < 0 && sy > 0) { ux = -o.x - o.y; uy = o.x - o.y; }
    else { ux = o.y - o.x; uy = -o.x - o.y; }
    x0 = {fmad<T>(h, ux, e.x), fmad<T>(h, uy, e.y)};
    x1 = {fmad<T>(-h, ux, e.x), fmad<T>(-h, uy, e.y)};
  } else {
    constexpr double c = cs2pi(k, R, 0);
    constexpr double s = DIR > 0 ? cs2pi(k, R, 1) : -cs2pi(k, R, 1);
    constexpr bool cosf = (c < 0 ? -c : c) >= (s < 0 ? -s : s);
    if constexpr (cosf) {
      // w o = c (o.x - t o.y, o.y + t o.x)
      constexpr T m = T(c), tq = T(s / c);
      const T ux = fmad<T>(-tq, o.y, o.x), uy = fmad<T>(tq, o.x, o.y);
      x0 = {fmad<T>(m, ux, e.x), fmad<T>(m, uy, e.y)};
      x1 = {fmad<T>(-m, ux, e.x), fmad<T>(-m, uy, e.y)};
    } else {
      // w o = s (t o.x - o.y, t o.y + o.x), t = c / s
      constexpr T m = T(s), tq = T(c / s);
      const T ux = fmad<T>(tq, o.x, -o.y), uy = fmad<T>(tq, o.y, o.x);
      x0 = {fmad<T>(m, ux, e.x), fmad<T>(m, uy, e.y)};
      x1 = {fmad<T>(-m, ux, e.x), fmad<T>(-m, uy, e.y)};
    }
  }
}

// In-register DFT of size R on v[0..R) (natural order in and out):
//   V[k] = sum_j v[j] exp(DIR * 2 pi i j k / R).
// Recursive radix-2 decimation in time; every index and twiddle is a
// compile-time constant, so the array lives in registers.
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    const cx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const cx<T> a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    const cx<T> b0 = cadd(v[1], v[3]), b1 = rot<1, 4, DIR>(csub(v[1], v[3]));
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, b1);
    v[3] = csub(a1, b1);
  } else {
    cx<T> e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    dft<R / 2, DIR, T>(e);
    dft<R / 2, DIR, T>(o);
    static_for<R / 2>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      bfly<k, R, DIR, T>(e[k], o[k], v[k], v[k + R / 2]);
    });
  }
}

// ------------------------------------------------------------------------
// Raw buffer access (MUBUF).  One resource per row, a per-lane byte offset in
// a VGPR and the per-register part of the offset as a uniform soffset: the
// loads of a thread's 32 elements then share one address register.  Offsets
// beyond the resource's byte count read as zero instead of faulting.
using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename V>
__device__ __forceinline__ V buf_load(rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(V) == 4) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  } else if constexpr (sizeof(V) == 8) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  } else {
    static_assert(sizeof(V) == 16, "buffer load width");
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  }
}

template <typename V>
__device__ __forceinline__ void buf_store(V v, rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(V) == 8) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
  } else {
    static_assert(sizeof(V) == 16, "buffer store width");
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff, soff, 0);
  }
}

// ------------------------------------------------------------------------
// Cross-half lane exchange.  v_permlane32_swap(D, S) swaps the upper 32
// lanes of D with the lower 32 lanes of S, i.e. D' = {D.lo, S.lo},
// S' = {D.hi, S.hi}.  Applied to (a, b) and then to (S', D') it yields
// {a.hi, a.lo} and {b.hi, b.lo}: each register with its halves exchanged,
// which is the value lane l ^ 32 holds.  Two swaps serve two registers.
__device__ __forceinline__ void halfswap2(uint32_t a, uint32_t b, uint32_t& sa, uint32_t& sb) {
  const auto r1 = __builtin_amdgcn_permlane32_swap(a, b, false, false);
  const auto r2 = __builtin_amdgcn_permlane32_swap(r1[1], r1[0], false, false);
  sa = r2[0];
  sb = r2[1];
}
// Per-lane blend: the lanes set in the constant mask take b, the others a.
// One v_cndmask per register with the mask in an SGPR pair (written in asm:
// the compiler turns such selects on single lanes into exec-masked branches).
__device__ __forceinline__ uint32_t lane_sel(uint64_t mask, uint32_t a, uint32_t b) {
  uint32_t r;
  asm volatile("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(mask));
  return r;
}
template <typename T>
__device__ __forceinline__ cx<T> lane_sel(uint64_t mask, const cx<T>& a, const cx<T>& b) {
  constexpr int W = sizeof(cx<T>) / 4;
  using V = typename std::conditional<W == 2, u32x2, u32x4>::type;
  const V ua = __builtin_bit_cast(V, a), ub = __builtin_bit_cast(V, b);
  V r;
#pragma unroll
  for (int i = 0; i < W; ++i) r[i] = lane_sel(mask, ua[i], ub[i]);
  return __builtin_bit_cast(cx<T>, r);
}

// a as held by lane l ^ 32 (complex, any real type; one swap per register)
template <typename T>
__device__ __forceinline__ cx<T> halfrot(const cx<T>& a) {
  constexpr int W = sizeof(cx<T>) / 4;
  using V = typename std::conditional<W == 2, u32x2, u32x4>::type;
  const V u = __builtin_bit_cast(V, a);
  V s;
#pragma unroll
  for (int i = 0; i < W; i += 2) {
    uint32_t x, y;
    halfswap2(u[i], u[i + 1], x, y);
    s[i] = x;
    s[i + 1] = y;
  }
  return __builtin_bit_cast(cx<T>, s);
}

// pa = b and pb = a as held by lane l ^ 32 (complex, any real type)
template <typename T>
__device__ __forceinline__ void partner_pair(const cx<T>& a, const cx<T>& b, cx<T>& pa, cx<T>& pb) {
  constexpr int W = sizeof(cx<T>) / 4;
  const auto ua = __builtin_bit_cast(typename std::conditional<W == 2, u32x2, u32x4>::type, a);
  const auto ub = __builtin_bit_cast(typename std::conditional<W == 2, u32x2, u32x4>::type, b);
  typename std::conditional<W == 2, u32x2, u32x4>::type sa, sb;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    uint32_t x, y;
    halfswap2(ua[i], ub[i], x, y);
    sa[i] = x;
    sb[i] = y;
  }
  pb = __builtin_bit_cast(cx<T>, sa);
  pa = __builtin_bit_cast(cx<T>, sb);
}

// ------------------------------------------------------------------------
// Wave64 helpers.
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// ------------------------------------------------------------------------
// Template spectrum storage formats.  All are loaded as cx<float>/cx<double>.
struct bf16x2 {
  uint16_t x, y;
};

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float(uint32_t(b) << 16);
}
// round to nearest even; NaN stays NaN
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return uint16_t((u >> 16) | 0x40u);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return uint16_t(u >> 16);
}

template <typename TW, typename T>
__device__ __forceinline__ cx<T> load_spec(const TW* p, uint32_t k) {
  if constexpr (std::is_same_v<TW, cx<T>>) {
    return p[k];
  } else if constexpr (std::is_same_v<TW, __half2>) {
    const float2 f = __half22float2(p[k]);
    return {f.x, f.y};
  } else {
    static_assert(std::is_same_v<TW, bf16x2>, "unknown spectrum storage");
    const bf16x2 b = p[k];
    return {bf16_to_f32(b.x), bf16_to_f32(b.y)};
  }
}

template <typename TW, typename T>
__device__ __forceinline__ void store_spec(TW* p, uint32_t k, cx<T> v) {
  if constexpr (std::is_same_v<TW, cx<T>>) {
    p[k] = v;
  } else if constexpr (std::is_same_v<TW, __half2>) {
    p[k] = __floats2half2_rn(float(v.x), float(v.y));
  } else {
    p[k] = bf16x2{f32_to_bf16(float(v.x)), f32_to_bf16(float(v.y))};
  }
}

}  // namespace bfs
