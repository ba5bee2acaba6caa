// Packed storage formats of the two-link field and of colour vectors.
//
// Every field is a set of planes; a plane holds one fixed-width word per site
// (sites in [z][y][x] order, plane length Vp), so a wavefront reading 64
// consecutive sites of a plane issues one fully coalesced vector load.
// Reals are kept in the order (re0, im0, re1, im1, ...): for a 3x3 matrix
// element k = 3a + b, for a colour vector component c.
//
//   precision  two-link field per site and direction        colour vector per site
//   FP64       9 planes double2 (one complex each)   144 B   3 planes double2      48 B
//   FP32       4 planes float4 + 1 plane float2        72 B   float4 + float2       24 B
//   F16S       2 planes 8 x half + 1 plane            40 B   1 plane: 6 x half     16 B
//              (2 x half, FP32 scale)                        + FP32 scale
//   BF16       2 planes 8 x bf16 + 1 plane 2 x bf16   36 B   4 x bf16 + 2 x bf16   12 B
//
// Twelve-real two-link forms (format code = precision | W12): only the first
// two rows of each matrix are stored and the third is rebuilt on load as the
// complex conjugate of the cross product of the first two, which is the third
// row of any SU(3) matrix (a two-link is a product of two SU(3) links):
//   FP64|W12   6 planes double2                        96 B
//   FP32|W12   3 planes float4                         48 B
//   F16S|W12   1 plane 8 x half + 1 plane 4 x half     24 B   (no scale: every entry
//   BF16|W12   1 plane 8 x bf16 + 1 plane 4 x bf16     24 B    of an SU(3) matrix is <= 1)
// Colour vectors keep the format of the precision.
//
// F16S stores value / s as IEEE half, with s = max |real| of the site (one
// scale per site and direction for W, per site and RHS for vectors); s = 0
// encodes an all-zero site.  Stores round to nearest even.  Vector quotients
// are formed as v * RN(1/s) in FP32, rounded to FP32 and then to half (with v
// and s pre-multiplied by 2^64 when s is subnormal); two-link quotients as
// v * (1/s) in FP64, rounded once to half.  The 16-bit twelve-real rows are
// rounded once from FP64 to half; FP64 values headed for bf16 are rounded to
// FP32 first.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "tl_internal.h"

namespace tl {

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ float bf16_to_f32(uint32_t bits16) { return __uint_as_float(bits16 << 16); }


__device__ __forceinline__ float h_to_f32(uint32_t bits16) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)bits16);
}


// FP64 -> half in one rounding (to nearest even).
__device__ __forceinline__ uint32_t f64_to_h(double d) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)d);
}

typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

// Two FP32 values to bf16 (round to nearest even) in one word, lo in bits 0-15: one
// v_cvt_pk_bf16_f32 on gfx950.
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f2){lo, hi}, v2bf));
}
// Two FP32 values to IEEE half (round to nearest even) in one word: one v_cvt_pk_f16_f32.
__device__ __forceinline__ uint32_t pack_h(float lo, float hi) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f2){lo, hi}, h2));
}
// Two-link reals (FP64): half in one rounding; bf16 through FP32.
__device__ __forceinline__ uint32_t pack_h_d(double lo, double hi) { return f64_to_h(lo) | (f64_to_h(hi) << 16); }
__device__ __forceinline__ uint32_t pack_bf16_d(double lo, double hi) { return pack_bf16((float)lo, (float)hi); }

// FP32 product rounded to FP32.  The empty asm makes the rounded product a value the
// compiler has to materialise: a product that is then converted to half would otherwise
// be fused with the conversion into one mixed-precision FMA (v_fma_mixlo_f16), which
// rounds once, to half -- not the vector format's definition (FP32 quotient, then half).
__device__ __forceinline__ float mul_f32(float a, float b) {
  float p = a * b;
  asm("" : "+v"(p));
  return p;
}

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef uint32_t v2u __attribute__((ext_vector_type(2)));

// One F16S colour vector: the six reals as half quotients q = v / s, s = max |v| (FP32),
// each q formed as v * (1/s) in FP32 and rounded to FP32, then to half.  A site whose
// maximum is an FP32 subnormal is first multiplied by 2^64 (exact), so that 1/s cannot
// overflow.  Returns the word (three half pairs, then the scale's bits) every store of
// the format writes and every load reads.
template <typename T>
__device__ __forceinline__ v4u f16s_encode(const T (&v)[6]) {
  float f[6];
  float mx = 0.0f;
#pragma unroll
  for (int c = 0; c < 6; c++) {
    f[c] = (float)v[c];
    mx = fmaxf(mx, fabsf(f[c]));
  }
  const float pre = mx < 1.17549435e-38f ? 18446744073709551616.0f : 1.0f;
  const float inv = mx > 0.0f ? 1.0f / (mx * pre) : 0.0f;
#pragma unroll
  for (int c = 0; c < 6; c++) f[c] = mul_f32(f[c] * pre, inv);
  return v4u{pack_h(f[0], f[1]), pack_h(f[2], f[3]), pack_h(f[4], f[5]), __float_as_uint(mx)};
}
// Its decoding: each half times the scale, rounded to FP32.
template <typename T>
__device__ __forceinline__ void f16s_decode(const v4u p, T (&v)[6]) {
  const float s = __uint_as_float(p.w);
  v[0] = h_to_f32(p.x & 0xffffu) * s; v[1] = h_to_f32(p.x >> 16) * s;
  v[2] = h_to_f32(p.y & 0xffffu) * s; v[3] = h_to_f32(p.y >> 16) * s;
  v[4] = h_to_f32(p.z & 0xffffu) * s; v[5] = h_to_f32(p.z >> 16) * s;
}

// Store one word; NT = nontemporal (streamed past the caches: the smearing step's
// output is not read again until the next step, long after it would be evicted).
template <bool NT, typename V>
__device__ __forceinline__ void put(V* p, V v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Third row of a special unitary 3x3 matrix from its first two rows (m[0..11]):
// m(2, k) = conj(m(0, j) m(1, l) - m(0, l) m(1, j)) for (k, j, l) cyclic.  The
// operation order is fixed, so every kernel rebuilds the same bits.
template <typename T>
__device__ __forceinline__ void su3_row3(T (&m)[18]) {
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const int j = (k + 1) % 3, l = (k + 2) % 3;
    const T ajr = m[2 * j], aji = m[2 * j + 1], alr = m[2 * l], ali = m[2 * l + 1];
    const T bjr = m[6 + 2 * j], bji = m[6 + 2 * j + 1], blr = m[6 + 2 * l], bli = m[6 + 2 * l + 1];
    T re = ajr * blr;
    re = fma_(-aji, bli, re);
    re = fma_(-alr, bjr, re);
    re = fma_(ali, bji, re);
    T im = ajr * bli;
    im = fma_(aji, blr, im);
    im = fma_(-alr, bji, im);
    im = fma_(-ali, bjr, im);
    m[12 + 2 * k] = re;
    m[12 + 2 * k + 1] = -im;
  }
}

// Load a word of a packed field through a global-address-space pointer.  The
// field pointers come from work-list entries in memory, whose address space
// the compiler cannot infer: plain dereferences would compile to flat loads,
// which also count against the LDS wait counter, so that every wait for LDS
// data (at a barrier) would wait for these loads too.
template <typename V>
__device__ __forceinline__ V ldg(const char* p) {
  return *(const __attribute__((address_space(1))) V*)p;
}

// Codes with the ONE bit store their (one-)link field exactly like code & 7.
template <int P> struct Fmt : Fmt<P & 7> {};

// ------------------------------------------------------------------ FP64
template <> struct Fmt<F64> {
  using real = double;
  template <typename T>
  __device__ static void load_w(const char* __restrict__ b, int64_t Vp, int64_t i, T (&m)[18]) {
#pragma unroll
    for (int k = 0; k < 9; k++) {
      const v2d v = ldg<v2d>(b + (k * Vp + i) * 16);
      m[2 * k] = (T)v.x;
      m[2 * k + 1] = (T)v.y;
    }
  }
  __device__ static void store_w(char* __restrict__ b, int64_t Vp, int64_t i, const double (&m)[18]) {
    v2d* p = reinterpret_cast<v2d*>(b);
#pragma unroll
    for (int k = 0; k < 9; k++) put<false>(p + k * Vp + i, v2d{m[2 * k], m[2 * k + 1]});
  }
  template <typename T>
  __device__ static void load_v(const char* __restrict__ b, int64_t Vp, int64_t i, T (&v)[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const v2d w = ldg<v2d>(b + (c * Vp + i) * 16);
      v[2 * c] = (T)w.x;
      v[2 * c + 1] = (T)w.y;
    }
  }
  template <typename T, bool NT = false>
  __device__ static void store_v(char* __restrict__ b, int64_t Vp, int64_t i, const T (&v)[6]) {
    v2d* p = reinterpret_cast<v2d*>(b);
#pragma unroll
    for (int c = 0; c < 3; c++) put<NT>(p + c * Vp + i, v2d{(double)v[2 * c], (double)v[2 * c + 1]});
  }
};

// ------------------------------------------------------------------ FP32
template <> struct Fmt<F32> {
  using real = float;
  template <typename T>
  __device__ static void load_w(const char* __restrict__ b, int64_t Vp, int64_t i, T (&m)[18]) {
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const v4f v = ldg<v4f>(b + (k * Vp + i) * 16);
      m[4 * k] = v.x;
      m[4 * k + 1] = v.y;
      m[4 * k + 2] = v.z;
      m[4 * k + 3] = v.w;
    }
    const v2f v = ldg<v2f>(b + 64 * Vp + i * 8);
    m[16] = v.x;
    m[17] = v.y;
  }
  __device__ static void store_w(char* __restrict__ b, int64_t Vp, int64_t i, const double (&m)[18]) {
    v4f* p = reinterpret_cast<v4f*>(b);
#pragma unroll
    for (int k = 0; k < 4; k++)
      put<false>(p + k * Vp + i, v4f{(float)m[4 * k], (float)m[4 * k + 1], (float)m[4 * k + 2], (float)m[4 * k + 3]});
    put<false>(reinterpret_cast<v2f*>(b + 64 * Vp) + i, v2f{(float)m[16], (float)m[17]});
  }
  template <typename T>
  __device__ static void load_v(const char* __restrict__ b, int64_t Vp, int64_t i, T (&v)[6]) {
    const v4f a = ldg<v4f>(b + i * 16);
    const v2f c = ldg<v2f>(b + 16 * Vp + i * 8);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = c.x; v[5] = c.y;
  }
  template <typename T, bool NT = false>
  __device__ static void store_v(char* __restrict__ b, int64_t Vp, int64_t i, const T (&v)[6]) {
    put<NT>(reinterpret_cast<v4f*>(b) + i, v4f{(float)v[0], (float)v[1], (float)v[2], (float)v[3]});
    put<NT>(reinterpret_cast<v2f*>(b + 16 * Vp) + i, v2f{(float)v[4], (float)v[5]});
  }
};

// ------------------------------------------------------------------ F16S
template <> struct Fmt<F16S> {
  using real = float;
  template <typename T>
  __device__ static void load_w(const char* __restrict__ b, int64_t Vp, int64_t i, T (&m)[18]) {
    const v4u p0 = ldg<v4u>(b + i * 16);
    const v4u p1 = ldg<v4u>(b + 16 * Vp + i * 16);
    const v2u p2 = ldg<v2u>(b + 32 * Vp + i * 8);
    const float s = __uint_as_float(p2.y);
    const uint32_t w[9] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w, p2.x};
#pragma unroll
    for (int k = 0; k < 9; k++) {
      m[2 * k] = h_to_f32(w[k] & 0xffffu) * s;
      m[2 * k + 1] = h_to_f32(w[k] >> 16) * s;
    }
  }
  __device__ static void store_w(char* __restrict__ b, int64_t Vp, int64_t i, const double (&m)[18]) {
    double mx = 0.0;
#pragma unroll
    for (int k = 0; k < 18; k++) mx = fmax(mx, fabs(m[k]));
    const float s = (float)mx;
    const double inv = s > 0.0f ? 1.0 / (double)s : 0.0;
    uint32_t w[9];
#pragma unroll
    for (int k = 0; k < 9; k++) w[k] = pack_h_d(m[2 * k] * inv, m[2 * k + 1] * inv);
    put<false>(reinterpret_cast<v4u*>(b) + i, v4u{w[0], w[1], w[2], w[3]});
    put<false>(reinterpret_cast<v4u*>(b + 16 * Vp) + i, v4u{w[4], w[5], w[6], w[7]});
    put<false>(reinterpret_cast<v2u*>(b + 32 * Vp) + i, v2u{w[8], __float_as_uint(s)});
  }
  template <typename T>
  __device__ static void load_v(const char* __restrict__ b, int64_t Vp, int64_t i, T (&v)[6]) {
    (void)Vp;
    f16s_decode(ldg<v4u>(b + i * 16), v);
  }
  template <typename T, bool NT = false>
  __device__ static void store_v(char* __restrict__ b, int64_t Vp, int64_t i, const T (&v)[6]) {
    (void)Vp;
    put<NT>(reinterpret_cast<v4u*>(b) + i, f16s_encode(v));
  }
};

// ------------------------------------------------------------------ BF16
template <> struct Fmt<BF16> {
  using real = float;
  template <typename T>
  __device__ static void load_w(const char* __restrict__ b, int64_t Vp, int64_t i, T (&m)[18]) {
    const v4u p0 = ldg<v4u>(b + i * 16);
    const v4u p1 = ldg<v4u>(b + 16 * Vp + i * 16);
    const uint32_t p2 = ldg<uint32_t>(b + 32 * Vp + i * 4);
    const uint32_t w[9] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w, p2};
#pragma unroll
    for (int k = 0; k < 9; k++) {
      m[2 * k] = bf16_to_f32(w[k] & 0xffffu);
      m[2 * k + 1] = bf16_to_f32(w[k] >> 16);
    }
  }
  __device__ static void store_w(char* __restrict__ b, int64_t Vp, int64_t i, const double (&m)[18]) {
    uint32_t w[9];
#pragma unroll
    for (int k = 0; k < 9; k++) w[k] = pack_bf16((float)m[2 * k], (float)m[2 * k + 1]);
    put<false>(reinterpret_cast<v4u*>(b) + i, v4u{w[0], w[1], w[2], w[3]});
    put<false>(reinterpret_cast<v4u*>(b + 16 * Vp) + i, v4u{w[4], w[5], w[6], w[7]});
    put<false>(reinterpret_cast<uint32_t*>(b + 32 * Vp) + i, w[8]);
  }
  template <typename T>
  __device__ static void load_v(const char* __restrict__ b, int64_t Vp, int64_t i, T (&v)[6]) {
    const v2u p = ldg<v2u>(b + i * 8);
    const uint32_t q = ldg<uint32_t>(b + 8 * Vp + i * 4);
    v[0] = bf16_to_f32(p.x & 0xffffu); v[1] = bf16_to_f32(p.x >> 16);
    v[2] = bf16_to_f32(p.y & 0xffffu); v[3] = bf16_to_f32(p.y >> 16);
    v[4] = bf16_to_f32(q & 0xffffu);   v[5] = bf16_to_f32(q >> 16);
  }
  template <typename T, bool NT = false>
  __device__ static void store_v(char* __restrict__ b, int64_t Vp, int64_t i, const T (&v)[6]) {
    put<NT>(reinterpret_cast<v2u*>(b) + i, v2u{pack_bf16((float)v[0], (float)v[1]), pack_bf16((float)v[2], (float)v[3])});
    put<NT>(reinterpret_cast<uint32_t*>(b + 8 * Vp) + i, pack_bf16((float)v[4], (float)v[5]));
  }
};

// ------------------------------------------------------------------ twelve-real two-links

template <> struct Fmt<F64 | W12> : Fmt<F64> {
  template <typename T>
  __device__ static void load_w(const char* __restrict__ b, int64_t Vp, int64_t i, T (&m)[18]) {
#pragma unroll
    for (int k = 0; k < 6; k++) {
      const v2d v = ldg<v2d>(b + (k * Vp + i) * 16);
      m[2 * k] = (T)v.x;
      m[2 * k + 1] = (T)v.y;
    }
    su3_row3(m);
  }
  __device__ static void store_w(char* __restrict__ b, int64_t Vp, int64_t i, const double (&m)[18]) {
    v2d* p = reinterpret_cast<v2d*>(b);
#pragma unroll
    for (int k = 0; k < 6; k++) put<false>(p + k * Vp + i, v2d{m[2 * k], m[2 * k + 1]});
  }
};

template <> struct Fmt<F32 | W12> : Fmt<F32> {
  template <typename T>
  __device__ static void load_w(const char* __restrict__ b, int64_t Vp, int64_t i, T (&m)[18]) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const v4f v = ldg<v4f>(b + (k * Vp + i) * 16);
      m[4 * k] = v.x;
      m[4 * k + 1] = v.y;
      m[4 * k + 2] = v.z;
      m[4 * k + 3] = v.w;
    }
    su3_row3(m);
  }
  __device__ static void store_w(char* __restrict__ b, int64_t Vp, int64_t i, const double (&m)[18]) {
    v4f* p = reinterpret_cast<v4f*>(b);
#pragma unroll
    for (int k = 0; k < 3; k++)
      put<false>(p + k * Vp + i, v4f{(float)m[4 * k], (float)m[4 * k + 1], (float)m[4 * k + 2], (float)m[4 * k + 3]});
  }
};

// 16-bit twelve-real forms: twelve values in a 16-byte and an 8-byte plane.
template <uint32_t (*Pack)(double, double), float (*Unpack)(uint32_t)>
struct Fmt16W12 {
  template <typename T>
  __device__ static void load_w(const char* __restrict__ b, int64_t Vp, int64_t i, T (&m)[18]) {
    const v4u p0 = ldg<v4u>(b + i * 16);
    const v2u p1 = ldg<v2u>(b + 16 * Vp + i * 8);
    const uint32_t w[6] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y};
#pragma unroll
    for (int k = 0; k < 6; k++) {
      m[2 * k] = Unpack(w[k] & 0xffffu);
      m[2 * k + 1] = Unpack(w[k] >> 16);
    }
    su3_row3(m);
  }
  __device__ static void store_w(char* __restrict__ b, int64_t Vp, int64_t i, const double (&m)[18]) {
    uint32_t w[6];
#pragma unroll
    for (int k = 0; k < 6; k++) w[k] = Pack(m[2 * k], m[2 * k + 1]);
    put<false>(reinterpret_cast<v4u*>(b) + i, v4u{w[0], w[1], w[2], w[3]});
    put<false>(reinterpret_cast<v2u*>(b + 16 * Vp) + i, v2u{w[4], w[5]});
  }
};

template <> struct Fmt<F16S | W12> : Fmt<F16S> {
  using W = Fmt16W12<pack_h_d, h_to_f32>;
  template <typename T>
  __device__ static void load_w(const char* __restrict__ b, int64_t Vp, int64_t i, T (&m)[18]) { W::load_w(b, Vp, i, m); }
  __device__ static void store_w(char* __restrict__ b, int64_t Vp, int64_t i, const double (&m)[18]) { W::store_w(b, Vp, i, m); }
};

template <> struct Fmt<BF16 | W12> : Fmt<BF16> {
  using W = Fmt16W12<pack_bf16_d, bf16_to_f32>;
  template <typename T>
  __device__ static void load_w(const char* __restrict__ b, int64_t Vp, int64_t i, T (&m)[18]) { W::load_w(b, Vp, i, m); }
  __device__ static void store_w(char* __restrict__ b, int64_t Vp, int64_t i, const double (&m)[18]) { W::store_w(b, Vp, i, m); }
};

// ------------------------------------------------------------------ plane pointers
// The same formats addressed through per-plane base pointers computed once per
// tile: every load is then a uniform 64-bit base plus a 32-bit site offset
// (site indices are below 2^27), which the compiler turns into scalar-base +
// vector-offset loads with no per-load 64-bit arithmetic.
// load_w_raw + finish_w split a two-link load so that the arithmetic that
// completes it (the third row of a twelve-real form) can be placed after a
// barrier; for the eighteen-real forms finish_w does nothing.

template <int P> struct Planes : Planes<P & 7> {};

template <class D, int NW_>
struct FullW {
  template <typename T>
  static __device__ __forceinline__ void load_w_raw(const char* const (&pl)[NW_], uint32_t i, T (&m)[18]) {
    D::load_w(pl, i, m);
  }
  template <typename T>
  static __device__ __forceinline__ void finish_w(T (&)[18]) {}
};

template <> struct Planes<F64> : FullW<Planes<F64>, 9> {
  static constexpr int NW = 9, NV = 3;
  static __device__ __forceinline__ void w(const char* b, int64_t Vp, const char* (&pl)[NW]) {
#pragma unroll
    for (int k = 0; k < 9; k++) pl[k] = b + 16 * Vp * k;
  }
  template <typename T>
  static __device__ __forceinline__ void load_w(const char* const (&pl)[NW], uint32_t i, T (&m)[18]) {
#pragma unroll
    for (int k = 0; k < 9; k++) {
      const v2d v = ldg<v2d>(pl[k] + i * 16u);
      m[2 * k] = (T)v.x;
      m[2 * k + 1] = (T)v.y;
    }
  }
  template <typename C>
  static __device__ __forceinline__ void v(C* b, int64_t Vp, C* (&pl)[NV]) {
#pragma unroll
    for (int k = 0; k < 3; k++) pl[k] = b + 16 * Vp * k;
  }
  template <typename T>
  static __device__ __forceinline__ void load_v(const char* const (&pl)[NV], uint32_t i, T (&v)[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const v2d w = ldg<v2d>(pl[c] + i * 16u);
      v[2 * c] = (T)w.x;
      v[2 * c + 1] = (T)w.y;
    }
  }
  template <typename T, bool NT>
  static __device__ __forceinline__ void store_v(char* const (&pl)[NV], uint32_t i, const T (&v)[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) put<NT>(reinterpret_cast<v2d*>(pl[c] + i * 16u), v2d{(double)v[2 * c], (double)v[2 * c + 1]});
  }
  // v <- what store_v followed by load_v would give back (the storage rounding, in registers)
  static __device__ __forceinline__ void round_v(double (&)[6]) {}
};

template <> struct Planes<F32> : FullW<Planes<F32>, 5> {
  static constexpr int NW = 5, NV = 2;
  static __device__ __forceinline__ void w(const char* b, int64_t Vp, const char* (&pl)[NW]) {
#pragma unroll
    for (int k = 0; k < 5; k++) pl[k] = b + 16 * Vp * k;
  }
  template <typename T>
  static __device__ __forceinline__ void load_w(const char* const (&pl)[NW], uint32_t i, T (&m)[18]) {
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const v4f v = ldg<v4f>(pl[k] + i * 16u);
      m[4 * k] = v.x;
      m[4 * k + 1] = v.y;
      m[4 * k + 2] = v.z;
      m[4 * k + 3] = v.w;
    }
    const v2f v = ldg<v2f>(pl[4] + i * 8u);
    m[16] = v.x;
    m[17] = v.y;
  }
  template <typename C>
  static __device__ __forceinline__ void v(C* b, int64_t Vp, C* (&pl)[NV]) {
    pl[0] = b;
    pl[1] = b + 16 * Vp;
  }
  template <typename T>
  static __device__ __forceinline__ void load_v(const char* const (&pl)[NV], uint32_t i, T (&v)[6]) {
    const v4f a = ldg<v4f>(pl[0] + i * 16u);
    const v2f c = ldg<v2f>(pl[1] + i * 8u);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = c.x; v[5] = c.y;
  }
  template <typename T, bool NT>
  static __device__ __forceinline__ void store_v(char* const (&pl)[NV], uint32_t i, const T (&v)[6]) {
    put<NT>(reinterpret_cast<v4f*>(pl[0] + i * 16u), v4f{(float)v[0], (float)v[1], (float)v[2], (float)v[3]});
    put<NT>(reinterpret_cast<v2f*>(pl[1] + i * 8u), v2f{(float)v[4], (float)v[5]});
  }
  static __device__ __forceinline__ void round_v(float (&)[6]) {}
};

template <> struct Planes<F16S> : FullW<Planes<F16S>, 3> {
  static constexpr int NW = 3, NV = 1;
  static __device__ __forceinline__ void w(const char* b, int64_t Vp, const char* (&pl)[NW]) {
    pl[0] = b;
    pl[1] = b + 16 * Vp;
    pl[2] = b + 32 * Vp;
  }
  template <typename T>
  static __device__ __forceinline__ void load_w(const char* const (&pl)[NW], uint32_t i, T (&m)[18]) {
    const v4u p0 = ldg<v4u>(pl[0] + i * 16u);
    const v4u p1 = ldg<v4u>(pl[1] + i * 16u);
    const v2u p2 = ldg<v2u>(pl[2] + i * 8u);
    const float s = __uint_as_float(p2.y);
    const uint32_t w[9] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w, p2.x};
#pragma unroll
    for (int k = 0; k < 9; k++) {
      m[2 * k] = h_to_f32(w[k] & 0xffffu) * s;
      m[2 * k + 1] = h_to_f32(w[k] >> 16) * s;
    }
  }
  template <typename C>
  static __device__ __forceinline__ void v(C* b, int64_t Vp, C* (&pl)[NV]) {
    (void)Vp;
    pl[0] = b;
  }
  template <typename T>
  static __device__ __forceinline__ void load_v(const char* const (&pl)[NV], uint32_t i, T (&v)[6]) {
    f16s_decode(ldg<v4u>(pl[0] + i * 16u), v);
  }
  template <typename T, bool NT>
  static __device__ __forceinline__ void store_v(char* const (&pl)[NV], uint32_t i, const T (&v)[6]) {
    put<NT>(reinterpret_cast<v4u*>(pl[0] + i * 16u), f16s_encode(v));
  }
  // the value a store and a reload of v give
  static __device__ __forceinline__ void round_v(float (&v)[6]) { f16s_decode(f16s_encode(v), v); }
};

template <> struct Planes<BF16> : FullW<Planes<BF16>, 3> {
  static constexpr int NW = 3, NV = 2;
  static __device__ __forceinline__ void w(const char* b, int64_t Vp, const char* (&pl)[NW]) {
    pl[0] = b;
    pl[1] = b + 16 * Vp;
    pl[2] = b + 32 * Vp;
  }
  template <typename T>
  static __device__ __forceinline__ void load_w(const char* const (&pl)[NW], uint32_t i, T (&m)[18]) {
    const v4u p0 = ldg<v4u>(pl[0] + i * 16u);
    const v4u p1 = ldg<v4u>(pl[1] + i * 16u);
    const uint32_t p2 = ldg<uint32_t>(pl[2] + i * 4u);
    const uint32_t w[9] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w, p2};
#pragma unroll
    for (int k = 0; k < 9; k++) {
      m[2 * k] = bf16_to_f32(w[k] & 0xffffu);
      m[2 * k + 1] = bf16_to_f32(w[k] >> 16);
    }
  }
  // Raw form: the nine packed words stay in m[0..8] (bit patterns) until finish_w
  // widens them, so a two-link loaded a step ahead holds nine registers, not 18.
  template <typename T>
  static __device__ __forceinline__ void load_w_raw(const char* const (&pl)[NW], uint32_t i, T (&m)[18]) {
    static_assert(sizeof(T) == 4, "BF16 two-links widen to FP32");
    const v4u p0 = ldg<v4u>(pl[0] + i * 16u);
    const v4u p1 = ldg<v4u>(pl[1] + i * 16u);
    const uint32_t p2 = ldg<uint32_t>(pl[2] + i * 4u);
    m[0] = __uint_as_float(p0.x); m[1] = __uint_as_float(p0.y); m[2] = __uint_as_float(p0.z);
    m[3] = __uint_as_float(p0.w); m[4] = __uint_as_float(p1.x); m[5] = __uint_as_float(p1.y);
    m[6] = __uint_as_float(p1.z); m[7] = __uint_as_float(p1.w); m[8] = __uint_as_float(p2);
  }
  // Widen in place from the last word down: word k fills m[2k] and m[2k+1], which
  // hold no word not yet read.
  template <typename T>
  static __device__ __forceinline__ void finish_w(T (&m)[18]) {
#pragma unroll
    for (int k = 8; k >= 0; k--) {
      const uint32_t w = __float_as_uint(m[k]);
      m[2 * k + 1] = bf16_to_f32(w >> 16);
      m[2 * k] = bf16_to_f32(w & 0xffffu);
    }
  }
  template <typename C>
  static __device__ __forceinline__ void v(C* b, int64_t Vp, C* (&pl)[NV]) {
    pl[0] = b;
    pl[1] = b + 8 * Vp;
  }
  template <typename T>
  static __device__ __forceinline__ void load_v(const char* const (&pl)[NV], uint32_t i, T (&v)[6]) {
    const v2u p = ldg<v2u>(pl[0] + i * 8u);
    const uint32_t q = ldg<uint32_t>(pl[1] + i * 4u);
    v[0] = bf16_to_f32(p.x & 0xffffu); v[1] = bf16_to_f32(p.x >> 16);
    v[2] = bf16_to_f32(p.y & 0xffffu); v[3] = bf16_to_f32(p.y >> 16);
    v[4] = bf16_to_f32(q & 0xffffu);   v[5] = bf16_to_f32(q >> 16);
  }
  template <typename T, bool NT>
  static __device__ __forceinline__ void store_v(char* const (&pl)[NV], uint32_t i, const T (&v)[6]) {
    put<NT>(reinterpret_cast<v2u*>(pl[0] + i * 8u), v2u{pack_bf16((float)v[0], (float)v[1]), pack_bf16((float)v[2], (float)v[3])});
    put<NT>(reinterpret_cast<uint32_t*>(pl[1] + i * 4u), pack_bf16((float)v[4], (float)v[5]));
  }
  static __device__ __forceinline__ void round_v(float (&v)[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const uint32_t w = pack_bf16(v[2 * c], v[2 * c + 1]);
      v[2 * c] = bf16_to_f32(w & 0xffffu);
      v[2 * c + 1] = bf16_to_f32(w >> 16);
    }
  }
};

// Twelve-real two-link forms: the plane pointers of rows 0 and 1.
template <class Base, int NW_>
struct PlanesW12 : Base {
  static constexpr int NW = NW_;
  static __device__ __forceinline__ void w(const char* b, int64_t Vp, const char* (&pl)[NW]) {
#pragma unroll
    for (int k = 0; k < NW; k++) pl[k] = b + 16 * Vp * k;
  }
  template <typename T>
  static __device__ __forceinline__ void finish_w(T (&m)[18]) { su3_row3(m); }
};

template <> struct Planes<F64 | W12> : PlanesW12<Planes<F64>, 6> {
  template <typename T>
  static __device__ __forceinline__ void load_w_raw(const char* const (&pl)[NW], uint32_t i, T (&m)[18]) {
#pragma unroll
    for (int k = 0; k < 6; k++) {
      const v2d v = ldg<v2d>(pl[k] + i * 16u);
      m[2 * k] = (T)v.x;
      m[2 * k + 1] = (T)v.y;
    }
  }
  template <typename T>
  static __device__ __forceinline__ void load_w(const char* const (&pl)[NW], uint32_t i, T (&m)[18]) {
    load_w_raw(pl, i, m);
    finish_w(m);
  }
};

template <> struct Planes<F32 | W12> : PlanesW12<Planes<F32>, 3> {
  template <typename T>
  static __device__ __forceinline__ void load_w_raw(const char* const (&pl)[NW], uint32_t i, T (&m)[18]) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const v4f v = ldg<v4f>(pl[k] + i * 16u);
      m[4 * k] = v.x;
      m[4 * k + 1] = v.y;
      m[4 * k + 2] = v.z;
      m[4 * k + 3] = v.w;
    }
  }
  template <typename T>
  static __device__ __forceinline__ void load_w(const char* const (&pl)[NW], uint32_t i, T (&m)[18]) {
    load_w_raw(pl, i, m);
    finish_w(m);
  }
};

template <class Base, float (*Unpack)(uint32_t)>
struct Planes16W12 : PlanesW12<Base, 2> {
  static constexpr int NW = 2;
  template <typename T>
  static __device__ __forceinline__ void load_w_raw(const char* const (&pl)[NW], uint32_t i, T (&m)[18]) {
    const v4u p0 = ldg<v4u>(pl[0] + i * 16u);
    const v2u p1 = ldg<v2u>(pl[1] + i * 8u);
    const uint32_t w[6] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y};
#pragma unroll
    for (int k = 0; k < 6; k++) {
      m[2 * k] = Unpack(w[k] & 0xffffu);
      m[2 * k + 1] = Unpack(w[k] >> 16);
    }
  }
  template <typename T>
  static __device__ __forceinline__ void load_w(const char* const (&pl)[NW], uint32_t i, T (&m)[18]) {
    load_w_raw(pl, i, m);
    PlanesW12<Base, 2>::finish_w(m);
  }
};

template <> struct Planes<F16S | W12> : Planes16W12<Planes<F16S>, h_to_f32> {};
template <> struct Planes<BF16 | W12> : Planes16W12<Planes<BF16>, bf16_to_f32> {};

}  // namespace tl
