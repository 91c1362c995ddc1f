// Device-side building blocks for the RTT kernels on gfx950 (CDNA4, wave64).
//
// Matrix-core formulation.  Every contraction step of the method multiplies
// a set of 1 x chi activation rows by one chi x chi core slice.  We compute
// the transpose, out^T = A^T x in^T, so that
//   * the MFMA "A" operand (M x K) is the core, M = output bond index,
//   * the MFMA "B" operand (K x N) holds the activations, N = 16 rows,
//   * the 16 x 16 result tile (M x N) gives 16 output features of 16 rows.
// Lane l of a wave works on row n = l % 16 and K-group g = l / 16.  For a
// row, group g owns the contiguous input features [g*chi/4, (g+1)*chi/4);
// core fragments are pre-swizzled on the host so that each lane's share of
// A is contiguous in memory.  Because lane l supplies the same K indices to A
// and B, the result does not depend on the order in which the hardware walks
// K inside one instruction.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rttk {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- BF16 bits
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);  // finite inputs only (activations are renormalised)
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}
// two FP32 values to a packed BF16 pair (element 0 in the low half), RNE,
// one hardware conversion
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b2 __attribute__((ext_vector_type(2)));
  const b2 h = __builtin_convertvector(f2{a, b}, b2);
  return __builtin_bit_cast(uint32_t, h);
}
// hi = RNE(x) and lo = RNE(x - hi) for a pair of values, packed
__device__ __forceinline__ void split_bf16x2(float a, float b, uint32_t& hi, uint32_t& lo) {
  hi = pack_bf16x2(a, b);
  lo = pack_bf16x2(a - __uint_as_float(hi << 16), b - __uint_as_float(hi & 0xffff0000u));
}

// ---------------------------------------------------------------- dtype traits
// Storage element of packed cores and the K-loop of one 16x16 output tile.
// prep() turns a lane's KPL FP32 activations into MFMA B operands once;
// mma() / mma2() run the K loop for one (or two, interleaved) core slices.
struct DF32 {
  using elem = float;
  static constexpr bool kF32 = true;  // FP32 activations on FP32 matrix ops
  template <int KPL>
  struct BOp { float v[KPL]; };
  template <int KPL>
  __device__ __forceinline__ static void prep(const float (&x)[KPL], BOp<KPL>& b) {
#pragma unroll
    for (int c = 0; c < KPL; ++c) b.v[c] = x[c];
  }
  template <int KPL>
  __device__ __forceinline__ static f4 mma(const float (&a)[KPL], const BOp<KPL>& b, f4 acc) {
#pragma unroll
    for (int c = 0; c < KPL; ++c)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[c], b.v[c], acc, 0, 0, 0);
    return acc;
  }
  template <int KPL>
  __device__ __forceinline__ static void mma2(const float (&a0)[KPL], const float (&a1)[KPL],
                                              const BOp<KPL>& b, f4& c0, f4& c1) {
#pragma unroll
    for (int c = 0; c < KPL; ++c) {
      c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[c], b.v[c], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[c], b.v[c], c1, 0, 0, 0);
    }
  }
  __device__ __forceinline__ static float to_f32(float x) { return x; }
};

// BF16 cores.  FP32 activations enter the matrix cores as a hi + lo BF16
// pair (two MFMAs), so each product keeps ~16 significant activation bits.
struct DBF16 {
  using elem = uint16_t;
  static constexpr bool kF32 = false;
  template <int KPL>
  struct BOp { bf16x8 hi[KPL / 8], lo[KPL / 8]; };
  template <int KPL>
  __device__ __forceinline__ static void prep(const float (&x)[KPL], BOp<KPL>& b) {
#pragma unroll
    for (int c = 0; c < KPL / 8; ++c) {
      uint4 h, l;
      split_bf16x2(x[8 * c + 0], x[8 * c + 1], h.x, l.x);
      split_bf16x2(x[8 * c + 2], x[8 * c + 3], h.y, l.y);
      split_bf16x2(x[8 * c + 4], x[8 * c + 5], h.z, l.z);
      split_bf16x2(x[8 * c + 6], x[8 * c + 7], h.w, l.w);
      b.hi[c] = __builtin_bit_cast(bf16x8, h);
      b.lo[c] = __builtin_bit_cast(bf16x8, l);
    }
  }
  template <int KPL>
  __device__ __forceinline__ static bf16x8 pack(const uint16_t (&a)[KPL], int c) {
    u16x8 av;
#pragma unroll
    for (int i = 0; i < 8; ++i) av[i] = a[8 * c + i];
    return __builtin_bit_cast(bf16x8, av);
  }
  template <int KPL>
  __device__ __forceinline__ static f4 mma(const uint16_t (&a)[KPL], const BOp<KPL>& b, f4 acc) {
#pragma unroll
    for (int c = 0; c < KPL / 8; ++c) {
      const bf16x8 av = pack<KPL>(a, c);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b.hi[c], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b.lo[c], acc, 0, 0, 0);
    }
    return acc;
  }
  template <int KPL>
  __device__ __forceinline__ static void mma2(const uint16_t (&a0)[KPL], const uint16_t (&a1)[KPL],
                                              const BOp<KPL>& b, f4& c0, f4& c1) {
#pragma unroll
    for (int c = 0; c < KPL / 8; ++c) {
      const bf16x8 x0 = pack<KPL>(a0, c), x1 = pack<KPL>(a1, c);
      c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, b.hi[c], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, b.hi[c], c1, 0, 0, 0);
      c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, b.lo[c], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, b.lo[c], c1, 0, 0, 0);
    }
  }
  __device__ __forceinline__ static float to_f32(uint16_t x) { return bf16_to_f32(x); }
};

// FP8 cores: one OCP e4m3 code per byte.  The matrix ops take a code c as
// the BF16 value c * 2^-9, decoded in registers by the gfx950 scaled
// conversion (exact: three mantissa bits, exponent well inside the BF16
// range).  Codes are at most 448 in magnitude, so the values the kernels see
// stay below 1 like the prescaled FP32 and BF16 cores; each position's
// exponent (FP8 scale + 9) is added back in the exponent bookkeeping.
// Activations are the hi + lo BF16 pair of DBF16.  Fragments stay FP8 in
// registers and are decoded where the matrix ops use them, so a fragment
// set takes half the registers of a BF16 one and half the bytes to load.
constexpr float kFp8Scale = 0.001953125f;  // 2^-9
struct DFP8 {
  using elem = uint8_t;
  static constexpr bool kF32 = false;
  // a lane's KPL codes decoded to BF16 bits (for fragments that serve many
  // matrix ops: decode once, then run them as BF16)
  template <int KPL>
  __device__ __forceinline__ static void decode(const uint8_t (&a)[KPL], uint16_t (&out)[KPL]);
  template <int KPL>
  using BOp = DBF16::BOp<KPL>;
  template <int KPL>
  __device__ __forceinline__ static void prep(const float (&x)[KPL], BOp<KPL>& b) {
    DBF16::prep<KPL>(x, b);
  }
  // the 8 codes at elements 8c .. 8c+7 of a lane's fragment as BF16 values
  template <int KPL>
  __device__ __forceinline__ static bf16x8 pack(const uint8_t (&a)[KPL], int c) {
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    uint32_t w0 = 0, w1 = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      w0 |= (uint32_t)a[8 * c + i] << (8 * i);
      w1 |= (uint32_t)a[8 * c + 4 + i] << (8 * i);
    }
    const b2 p0 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w0, kFp8Scale, false);
    const b2 p1 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w0, kFp8Scale, true);
    const b2 p2 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w1, kFp8Scale, false);
    const b2 p3 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w1, kFp8Scale, true);
    return bf16x8{p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
  }
  __device__ __forceinline__ static float to_f32(uint8_t x) {
    return (float)__builtin_amdgcn_cvt_scalef32_pk_bf16_fp8((uint32_t)x, kFp8Scale, false)[0];
  }
  template <int KPL>
  __device__ __forceinline__ static f4 mma(const uint8_t (&a)[KPL], const BOp<KPL>& b, f4 acc) {
#pragma unroll
    for (int c = 0; c < KPL / 8; ++c) {
      const bf16x8 av = pack<KPL>(a, c);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b.hi[c], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b.lo[c], acc, 0, 0, 0);
    }
    return acc;
  }
  template <int KPL>
  __device__ __forceinline__ static void mma2(const uint8_t (&a0)[KPL], const uint8_t (&a1)[KPL],
                                              const BOp<KPL>& b, f4& c0, f4& c1) {
#pragma unroll
    for (int c = 0; c < KPL / 8; ++c) {
      const bf16x8 x0 = pack<KPL>(a0, c), x1 = pack<KPL>(a1, c);
      c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, b.hi[c], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, b.hi[c], c1, 0, 0, 0);
      c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, b.lo[c], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, b.lo[c], c1, 0, 0, 0);
    }
  }
};

template <int KPL>
__device__ __forceinline__ void DFP8::decode(const uint8_t (&a)[KPL], uint16_t (&out)[KPL]) {
#pragma unroll
  for (int c = 0; c < KPL / 8; ++c) {
    const u16x8 v = __builtin_bit_cast(u16x8, pack<KPL>(a, c));
#pragma unroll
    for (int i = 0; i < 8; ++i) out[8 * c + i] = v[i];
  }
}

// Workgroup barrier that orders LDS only: global loads issued before it
// (prefetched core fragments) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Fragment tiles hold 64 lanes x KPL elements in 16-byte chunks, chunk-major:
// element e of lane l sits at ((e / CE) * 64 + l) * CE + e % CE, CE = 16 /
// element size.  One 16-byte load of the 64 lanes then reads 1 KB of
// consecutive bytes (8 cache lines) instead of touching 32 lines a quarter
// each, which is what limited the rate at which CUs take fragments from L2.
__host__ __device__ constexpr size_t frag_offset(int lane, int e, int ce) {
  return ((size_t)(e / ce) * 64 + lane) * ce + e % ce;
}
// chunk length in elements: 16 bytes, or a lane's whole fragment when that is
// shorter (FP8 at bond 32: 8 codes, one 8-byte load)
__host__ __device__ constexpr int frag_chunk(int elem_bytes, int kpl) {
  return 16 / elem_bytes < kpl ? 16 / elem_bytes : kpl;
}

// Load a lane's KPL-element fragment from a tile (16-byte aligned).
template <int KPL>
__device__ __forceinline__ void load_frag(float (&dst)[KPL], const float* tile, int lane) {
  const float4* s = reinterpret_cast<const float4*>(tile) + lane;
#pragma unroll
  for (int i = 0; i < KPL / 4; ++i) {
    float4 v = s[64 * i];
    dst[4 * i + 0] = v.x; dst[4 * i + 1] = v.y; dst[4 * i + 2] = v.z; dst[4 * i + 3] = v.w;
  }
}
template <int KPL>
__device__ __forceinline__ void load_frag(uint16_t (&dst)[KPL], const uint16_t* tile, int lane) {
  const uint4* s = reinterpret_cast<const uint4*>(tile) + lane;
#pragma unroll
  for (int i = 0; i < KPL / 8; ++i) {
    uint4 v = s[64 * i];
    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      dst[8 * i + 2 * j] = (uint16_t)(w[j] & 0xffffu);
      dst[8 * i + 2 * j + 1] = (uint16_t)(w[j] >> 16);
    }
  }
}

template <int KPL>
__device__ __forceinline__ void load_frag(uint8_t (&dst)[KPL], const uint8_t* tile, int lane) {
  if constexpr (KPL % 16 == 0) {
    const uint4* s = reinterpret_cast<const uint4*>(tile) + lane;
#pragma unroll
    for (int i = 0; i < KPL / 16; ++i) {
      uint4 v = s[64 * i];
      uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 16; ++j) dst[16 * i + j] = (uint8_t)(w[j / 4] >> (8 * (j % 4)));
    }
  } else {
    static_assert(KPL == 8, "FP8 fragments of 8 or a multiple of 16 codes per lane");
    const uint2 v = reinterpret_cast<const uint2*>(tile)[lane];
#pragma unroll
    for (int j = 0; j < 8; ++j) dst[j] = (uint8_t)((j < 4 ? v.x : v.y) >> (8 * (j % 4)));
  }
}

// Read KPL consecutive floats of LDS (16-byte aligned).
template <int KPL>
__device__ __forceinline__ void lds_read(float (&dst)[KPL], const float* src) {
  const float4* s = reinterpret_cast<const float4*>(src);
#pragma unroll
  for (int i = 0; i < KPL / 4; ++i) {
    float4 v = s[i];
    dst[4 * i + 0] = v.x; dst[4 * i + 1] = v.y; dst[4 * i + 2] = v.z; dst[4 * i + 3] = v.w;
  }
}

// Reductions over the four K-groups of a wave (lanes m, m+16, m+32, m+48)
// with the gfx950 lane-swap instructions (no LDS crossbar round trip).
__device__ __forceinline__ float group_max(float x) {
  const unsigned u = __float_as_uint(x);
  auto a = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  x = fmaxf(__uint_as_float(a[0]), __uint_as_float(a[1]));
  const unsigned v = __float_as_uint(x);
  auto b = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return fmaxf(__uint_as_float(b[0]), __uint_as_float(b[1]));
}
__device__ __forceinline__ float group_sum(float x) {
  const unsigned u = __float_as_uint(x);
  auto a = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  x = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  const unsigned v = __float_as_uint(x);
  auto b = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

// Max |x| over a row held by the four K-groups, then the power-of-two
// exponent e with max * 2^-e in [0.5, 1).  Scaling by 2^-e is exact, so
// renormalisation adds no rounding.
template <int KPL>
__device__ __forceinline__ int renorm_row(float (&v)[KPL]) {
  float mx = 0.f;
#pragma unroll
  for (int c = 0; c < KPL; ++c) mx = fmaxf(mx, fabsf(v[c]));
  mx = group_max(mx);
  int e = (mx > 0.f) ? __builtin_amdgcn_frexp_expf(mx) : 0;
#pragma unroll
  for (int c = 0; c < KPL; ++c) v[c] = __builtin_amdgcn_ldexpf(v[c], -e);
  return e;
}

// ---------------------------------------------------------------- activation rows
// Act<D, CHI> keeps a row of CHI activations in LDS in the form the matrix
// ops take, so that the wave producing a value converts it once instead of
// every consuming wave converting it again: FP32 values for FP32 cores; for
// BF16 cores the hi and lo BF16 parts, hi = RNE(x), lo = RNE(x - hi) (the
// same pair the MFMA would be fed from x).  Either way a row is CHI dwords
// (BF16: hi[0..CHI) then lo[0..CHI) as 16-bit words).
template <class D, int CHI>
struct Act;

template <int CHI>
struct Act<DF32, CHI> {
  template <int KPL>
  __device__ __forceinline__ static void load_b(const float* row, int g, DF32::BOp<KPL>& b) {
    lds_read<KPL>(b.v, row + g * KPL);
  }
  // exponent e of the row's largest |x| (all four K-groups), max * 2^-e in [0.5, 1)
  template <int KPL>
  __device__ __forceinline__ static int row_exp(const DF32::BOp<KPL>& b) {
    float mx = 0.f;
#pragma unroll
    for (int c = 0; c < KPL; ++c) mx = fmaxf(mx, fabsf(b.v[c]));
    mx = group_max(mx);
    return (mx > 0.f) ? __builtin_amdgcn_frexp_expf(mx) : 0;
  }
  template <int KPL>
  __device__ __forceinline__ static void load_f32(const float* row, int g, float (&v)[KPL]) {
    lds_read<KPL>(v, row + g * KPL);
  }
  __device__ __forceinline__ static void store4(float* row, int col, f4 v) {
    *reinterpret_cast<float4*>(row + col) = make_float4(v[0], v[1], v[2], v[3]);
  }
  __device__ __forceinline__ static void store1(float* row, int col, float x) { row[col] = x; }
  __device__ __forceinline__ static float get(const float* row, int i) { return row[i]; }
  __device__ __forceinline__ static void set_unit(float* row) { row[0] = 1.f; }
  // the first dword of a stored unit vector e_0 (the rest are zero)
  __device__ __forceinline__ static float unit_dword() { return 1.f; }
  // copy the four activations at col..col+3 of a row
  __device__ __forceinline__ static void copy4(float* dst, const float* src, int col) {
    *reinterpret_cast<float4*>(dst + col) = *reinterpret_cast<const float4*>(src + col);
  }
};

template <int CHI>
struct Act<DBF16, CHI> {
  __device__ __forceinline__ static const uint16_t* hi(const float* row) {
    return reinterpret_cast<const uint16_t*>(row);
  }
  __device__ __forceinline__ static uint16_t* hi(float* row) { return reinterpret_cast<uint16_t*>(row); }
  template <int KPL>
  __device__ __forceinline__ static void load_b(const float* row, int g, DBF16::BOp<KPL>& b) {
    const uint16_t* h = hi(row) + g * KPL;
#pragma unroll
    for (int c = 0; c < KPL / 8; ++c) {
      b.hi[c] = *reinterpret_cast<const bf16x8*>(h + 8 * c);
      b.lo[c] = *reinterpret_cast<const bf16x8*>(h + CHI + 8 * c);
    }
  }
  // the exponent is taken from the hi parts; any power of two is exact, and
  // every wave derives the same one from the same bits
  template <int KPL>
  __device__ __forceinline__ static int row_exp(const DBF16::BOp<KPL>& b) {
    uint32_t mx = 0;
#pragma unroll
    for (int c = 0; c < KPL / 8; ++c) {
      const u16x8 u = __builtin_bit_cast(u16x8, b.hi[c]);
#pragma unroll
      for (int i = 0; i < 8; ++i) mx = max(mx, (uint32_t)(u[i] & 0x7fffu));
    }
    const float f = group_max(__uint_as_float(mx << 16));
    return (f > 0.f) ? __builtin_amdgcn_frexp_expf(f) : 0;
  }
  template <int KPL>
  __device__ __forceinline__ static void load_f32(const float* row, int g, float (&v)[KPL]) {
    const uint16_t* h = hi(row) + g * KPL;
#pragma unroll
    for (int c = 0; c < KPL / 8; ++c) {
      const u16x8 a = *reinterpret_cast<const u16x8*>(h + 8 * c);
      const u16x8 l = *reinterpret_cast<const u16x8*>(h + CHI + 8 * c);
#pragma unroll
      for (int i = 0; i < 8; ++i) v[8 * c + i] = bf16_to_f32(a[i]) + bf16_to_f32(l[i]);
    }
  }
  __device__ __forceinline__ static void split(float x, uint16_t& h, uint16_t& l) {
    const __bf16 xh = (__bf16)x;  // round to nearest even
    const __bf16 xl = (__bf16)(x - (float)xh);
    h = __builtin_bit_cast(uint16_t, xh);
    l = __builtin_bit_cast(uint16_t, xl);
  }
  __device__ __forceinline__ static void store4(float* row, int col, f4 v) {
    uint32_t h01, l01, h23, l23;
    split_bf16x2(v[0], v[1], h01, l01);
    split_bf16x2(v[2], v[3], h23, l23);
    uint16_t* p = hi(row) + col;
    *reinterpret_cast<uint2*>(p) = make_uint2(h01, h23);
    *reinterpret_cast<uint2*>(p + CHI) = make_uint2(l01, l23);
  }
  // store4 through non-temporal stores (rows in global memory)
  __device__ __forceinline__ static void store4_nt(float* row, int col, f4 v) {
    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
    uint32_t h01, l01, h23, l23;
    split_bf16x2(v[0], v[1], h01, l01);
    split_bf16x2(v[2], v[3], h23, l23);
    uint16_t* p = hi(row) + col;
    __builtin_nontemporal_store(u2{h01, h23}, reinterpret_cast<u2*>(p));
    __builtin_nontemporal_store(u2{l01, l23}, reinterpret_cast<u2*>(p + CHI));
  }
  __device__ __forceinline__ static void store1(float* row, int col, float x) {
    uint16_t h, l;
    split(x, h, l);
    hi(row)[col] = h;
    hi(row)[CHI + col] = l;
  }
  __device__ __forceinline__ static float get(const float* row, int i) {
    return bf16_to_f32(hi(row)[i]) + bf16_to_f32(hi(row)[CHI + i]);
  }
  __device__ __forceinline__ static void set_unit(float* row) { hi(row)[0] = 0x3F80u; }
  // the first dword of a stored unit vector e_0: hi[0] = 1, hi[1] = 0
  __device__ __forceinline__ static float unit_dword() { return __uint_as_float(0x3F80u); }
  // copy the four activations at col..col+3 of a row (hi and lo parts)
  __device__ __forceinline__ static void copy4(float* dst, const float* src, int col) {
    *reinterpret_cast<uint2*>(hi(dst) + col) = *reinterpret_cast<const uint2*>(hi(src) + col);
    *reinterpret_cast<uint2*>(hi(dst) + CHI + col) = *reinterpret_cast<const uint2*>(hi(src) + CHI + col);
  }
};

// FP8 cores take the same activation rows as BF16 cores
template <int CHI>
struct Act<DFP8, CHI> : Act<DBF16, CHI> {};

// ---------------------------------------------------------------- Philox4x64-10
// Salmon et al., SC'11: 10 rounds of two 64x64->128 multiplies per block,
// key bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint64_t philox4x64_10_word0(uint64_t c0, uint64_t c1, uint64_t c2,
                                                         uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return c0;
}

__device__ __forceinline__ double philox_uniform(uint64_t seed, uint64_t stream, uint64_t walker,
                                                 uint64_t sweep, uint64_t spin) {
  uint64_t x = philox4x64_10_word0(walker, sweep, spin, 0, seed, stream);
  return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ int spin_bit(const uint64_t* words, int q) {
  return (int)((words[q >> 6] >> (q & 63)) & 1ull);
}

}  // namespace rttk
