// HIP kernels of the RTT Monte Carlo path (gfx950).
//
//  pass_kernel     one contraction pass of the flip-ratio schedule: the base
//                  environment vector plus one flipped vector per spin, all
//                  advanced core by core on the matrix cores (forward: row
//                  vectors from the left boundary to the cut bond; backward:
//                  column vectors from the right boundary to the cut).
//  combine_kernel  meets forward and backward vectors at the cut: amplitude,
//                  every single-flip ratio, linear-combination sums and the
//                  TFIM local energy, all in FP64.
//  chain_kernel    16 walkers per block as the 16 matrix-core columns:
//                  amplitudes (rows from the left and columns from the right
//                  meeting half way), and Metropolis sweeps with Philox uniforms.
//  reduce_kernel   compensated FP64 sums of local energies.
#pragma once
#include <float.h>
#include <math.h>

#include <type_traits>

#include "rtt_device.hpp"

namespace rttk {

constexpr int kMaxTerms = 8;
#ifndef PASS_PF_FP8
#define PASS_PF_FP8 2
#endif
#ifndef CHAIN_PF_FP8_256
#define CHAIN_PF_FP8_256 2
#endif
#ifndef CHAIN_SW_FP8_256
#define CHAIN_SW_FP8_256 2
#endif
// steps between power-of-two renormalisations: a row grows by at most chi
// per step, so 8 steps stay below 2^64 even at chi = 256 (FP32 range 2^128)
constexpr int kRenormEvery = 8;

template <int CHI>
struct Geo {
  static constexpr int WPW = CHI >= 64 ? 4 : CHI / 16;  // waves per walker / chain
  static constexpr int MT = CHI / (16 * WPW);           // 16-feature output tiles per wave
  static constexpr int KPL = CHI / 4;                   // input features per lane per row
  static constexpr int RS = CHI + 4;                    // LDS row stride (floats)
};

// ============================================================================
// pass kernel
// ============================================================================
// Schedule entry (int4): x = core position k, y = spin q read at k,
// z = active rows after this step, w = odd row (in | out << 16).  The odd row
// is the row of spin q: on the step where q first appears it is spawned from
// the base row (in = 0), otherwise it is q's own row (in = out).  It uses
// slice 1 - s_q; every other active row uses slice s_q.
struct PassArgs {
  const void* cores;        // [T][L][2][CHI*CHI], fragment layout of this direction
  const int32_t* core_exp;  // [T][L] power-of-two scale exponents, or null
  const int4* sched;        // schedules of all row groups, concatenated
  const int2* gsteps;       // [ng] (first entry, number of entries) of each group
  int ng;                   // row groups: spins are split so a group's rows fit on chip
  int nslot;                // rows per walker and group, multiple of 16
  int L, nw, W;
  const uint64_t* spins;    // [W][nw]
  float* out_vec;           // [T][ng][W][nslot][CHI]
  int32_t* out_exp;         // [T][ng][W][nslot]
};

// ----------------------------------------------------------------------------
// Flip-ratio pass with the K loop outermost (FP8 cores at bond 256, BF16 and
// FP8 cores at bond 128).  One walker per block; wave wv owns output
// features [wv chi / 4, (wv + 1) chi / 4), MT = chi / 64 tiles of 16.  For
// each 32-wide K chunk a lane's 8 core values of every tile are taken from
// its fragment word once (FP8 codes decoded to BF16), each active row tile's
// activations for that chunk are read from LDS once and multiplied into the
// MT tiles' accumulators, which stay live for the whole step.  Every
// accumulator sees the matrix-op sequence of pass_body (chunk by chunk, hi
// part then lo part), so the results are the same bits.
// With PASS_W_INPL rows are updated in place: the step's outputs wait in
// registers until every wave has read its inputs, so a walker's rows take
// half the LDS and twice as many fit (fewer row groups, fewer core reads).
// Tuning on the 16x16 four-term workload (local energies, 16384 walkers):
// the double-buffered item form 2.75 s; K outermost, two buffers 2.59 s; in
// place with 6 row tiles 2.22 s; with 9 (two row groups instead of three)
// and the two-slot ring below 2.06 s; with each step compiled for its exact
// row-tile count (no per-tile branches) 1.61 s, and for whether it
// renormalises (no scaling on the other steps) 1.55 s.  A four-slot ring
// spills.
#ifndef PASS_W_NTM  // row tiles a group may hold
#define PASS_W_NTM 9
#endif
#ifndef PASS_W_INPL
#define PASS_W_INPL 1
#endif
#ifndef PASS_W_ENABLE  // 0: every pass runs pass_body's item form
#define PASS_W_ENABLE 1
#endif
#ifndef PASS_W_RING  // fragment ring slots: 4 = one step ahead, 2 = half a step
#define PASS_W_RING 2
#endif
constexpr int kPassWideTiles = PASS_W_NTM;        // row tiles a step may hold
constexpr bool kPassWideInPlace = PASS_W_INPL != 0;

// PASS_W_128 also runs FP8 and BF16 at bond 128 in this form (bit-identical
// there), compiled for two waves per SIMD (pass_min_blocks): 10x10 bond-128
// BF16 local energies 18.7 -> 16.7 ms against the item form; left free to
// use one wave per SIMD it was slower (30.2 ms).  BF16 at bond 256 spills
// in this form.
#ifndef PASS_W_128
#define PASS_W_128 1
#endif
template <class D, int CHI>
constexpr bool pass_wide_form() {
  return PASS_W_ENABLE && ((std::is_same<D, DFP8>::value && (CHI == 256 || (PASS_W_128 && CHI == 128))) ||
                           (std::is_same<D, DBF16>::value && PASS_W_128 && CHI == 128));
}

// blocks per CU the pass kernels are compiled for (a register budget): two
// for the bond-128 K-outer form, whose registers would otherwise grow past
// what two waves per SIMD allow
template <class D, int CHI>
constexpr int pass_min_blocks() { return (pass_wide_form<D, CHI>() && CHI == 128) ? 2 : 1; }

template <class D, int CHI>
__device__ __forceinline__ void pass_body_wide(const PassArgs& a, int bx, int ty) {
  constexpr bool F8 = std::is_same<D, DFP8>::value;
  constexpr int KPL = CHI / 4, MT = CHI / 64, RS = CHI + 4, NTM = kPassWideTiles;
  constexpr int NCH = KPL / 8;     // 32-wide K chunks per step
  constexpr int CPW = F8 ? 2 : 1;  // K chunks per 16-byte fragment word (FP8: 16 codes)
  constexpr int NWD = NCH / CPW;   // fragment words per lane and tile
  static_assert(NTM >= 1 && NTM <= 9, "the step dispatch covers 1 to 9 row tiles");
  constexpr bool INPL = kPassWideInPlace;
  constexpr int NB = INPL ? 1 : 2;  // row buffers
  using A = Act<D, CHI>;
  using E = typename D::elem;
  extern __shared__ __align__(16) float lds[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, m = lane & 15;
  const int w = bx < a.W ? bx : a.W - 1;
  const int nslot = a.nslot;
  const int bufsz = nslot * RS;
  float* cur = lds;
  float* nxt = INPL ? lds : lds + bufsz;
  int* exc = reinterpret_cast<int*>(lds + NB * bufsz);
  int* exn = INPL ? exc : exc + nslot;
  uint64_t* spw = reinterpret_cast<uint64_t*>(lds + NB * bufsz + NB * nslot);
  for (int i = threadIdx.x; i < NB * bufsz; i += 256) cur[i] = 0.f;
  for (int i = threadIdx.x; i < NB * nslot; i += 256) exc[i] = 0;
  for (int i = threadIdx.x; i < a.nw; i += 256) spw[i] = a.spins[(size_t)w * a.nw + i];
  __syncthreads();
  if (threadIdx.x == 0) A::set_unit(cur);  // boundary vector e_0 in the base slot
  __syncthreads();

  const int term = ty / a.ng, grp = ty % a.ng;
  const E* cores = static_cast<const E*>(a.cores) + (size_t)term * a.L * 2 * CHI * CHI;
  const int* cexp_p = a.core_exp ? a.core_exp + (size_t)term * a.L : nullptr;
  const int2 gs = a.gsteps[grp];
  const int4* sched = a.sched + gs.x;
  const int n = gs.y;

  // Ring of fragment words: a slot holds one 16-byte word j of each lane's
  // fragment (elements 16j .. 16j + 15 for FP8 codes, 8j .. 8j + 7 for BF16)
  // of this wave's MT tiles, of the walker's slice (Rm) and, on steps with an
  // odd row, of the other slice (Ro).  A step streams its NWD words through
  // the RING slots; a slot is refilled with the word RING places further on
  // (in this step or the next) as soon as its K chunks are decoded, so every
  // load has RING / NWD of a step to arrive.
  constexpr int RING = PASS_W_RING < NWD ? PASS_W_RING : NWD;
  uint4 Rm[RING][MT], Ro[RING][MT];
  constexpr int TILE16 = 64 * KPL * (int)sizeof(E) / 16;  // 16-byte words per fragment tile
  // load word j of a step's fragments into ring slot j % RING
  auto issue = [&](int j, const int4& st, int bit) {
    const int sl = j % RING;
    const uint4* bm = reinterpret_cast<const uint4*>(cores + ((size_t)st.x * 2 + bit) * (CHI * CHI)) +
                      (size_t)wv * MT * TILE16;
#pragma unroll
    for (int q = 0; q < MT; ++q) Rm[sl][q] = bm[q * TILE16 + 64 * j + lane];
    if (st.w >= 0) {
      const uint4* bo = reinterpret_cast<const uint4*>(cores + ((size_t)st.x * 2 + (bit ^ 1)) * (CHI * CHI)) +
                        (size_t)wv * MT * TILE16;
#pragma unroll
      for (int q = 0; q < MT; ++q) Ro[sl][q] = bo[q * TILE16 + 64 * j + lane];
    }
  };
  // the A operand of K chunk c from its fragment word: FP8 codes 8c .. 8c + 7
  // (half h = c % 2 of the word) decoded to BF16, or the word's 8 BF16 values
  auto dec = [](const uint4& v, int h) -> bf16x8 {
    if constexpr (F8) {
      const uint32_t w0 = h ? v.z : v.x, w1 = h ? v.w : v.y;
      const auto p0 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w0, kFp8Scale, false);
      const auto p1 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w0, kFp8Scale, true);
      const auto p2 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w1, kFp8Scale, false);
      const auto p3 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w1, kFp8Scale, true);
      return bf16x8{p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
    } else {
      return __builtin_bit_cast(bf16x8, v);
    }
  };

  if (n > 0) {
    const int4 st0 = sched[0];
    const int bit0 = spin_bit(spw, st0.y);
#pragma unroll
    for (int j = 0; j < RING; ++j) issue(j, st0, bit0);
  }
  for (int s = 0; s < n; ++s) {
    const int4 st = sched[s];
    const int k = st.x, nact = st.z, odd = st.w;
    const int oin = odd >= 0 ? (odd & 0xffff) : -1, oout = odd >> 16;
    const int ot = odd >= 0 ? (oin >> 4) : -1;  // row tile of the odd row's input
    const int ntile = (nact + 15) >> 4;
    // renormalise every kRenormEvery steps (a row grows by at most chi per step)
    const bool rn = (s % kRenormEvery) == 0;
    const int4 stn = sched[min(s + 1, n - 1)];
    const int bitc = spin_bit(spw, st.y), bitn = spin_bit(spw, stn.y);
    const int cexp = cexp_p ? cexp_p[k] : 0;
    const float* orow = cur + (16 * (ot < 0 ? 0 : ot) + m) * RS;  // the odd row's input tile
    // One step over exactly NT row tiles (dispatched below on the step's
    // tile count): no branch per tile, so the compiler is free to issue a
    // chunk's reads ahead of the matrix ops, and no accumulator of an idle
    // tile is carried through the K loop.
    auto step = [&](auto ntc, auto rnc) {
      constexpr int NT = decltype(ntc)::value;
      constexpr bool RN = decltype(rnc)::value;  // a renormalisation step
      f4 acc[NT][MT], oacc[MT];
#pragma unroll
      for (int r = 0; r < NT; ++r) {
#pragma unroll
        for (int q = 0; q < MT; ++q) acc[r][q] = f4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int q = 0; q < MT; ++q) oacc[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int j = c / CPW, h = c % CPW, sl = j % RING;
        bf16x8 Am[MT];
#pragma unroll
        for (int q = 0; q < MT; ++q) Am[q] = dec(Rm[sl][q], h);
        // the odd row: the other slice applied to its input row (the same
        // LDS values its tile reads above)
        if (ot >= 0) {
          bf16x8 Ao[MT];
#pragma unroll
          for (int q = 0; q < MT; ++q) Ao[q] = dec(Ro[sl][q], h);
          const uint16_t* hp = A::hi(orow) + g * KPL + 8 * c;
          const bf16x8 bh = *reinterpret_cast<const bf16x8*>(hp);
          const bf16x8 bl = *reinterpret_cast<const bf16x8*>(hp + CHI);
#pragma unroll
          for (int q = 0; q < MT; ++q) {
            oacc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ao[q], bh, oacc[q], 0, 0, 0);
            oacc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ao[q], bl, oacc[q], 0, 0, 0);
          }
        }
        // the slot is free: refill it with the word RING places further on
        if (h == CPW - 1) {
          if (j + RING < NWD) issue(j + RING, st, bitc);
          else issue(j + RING - NWD, stn, bitn);
        }
#pragma unroll
        for (int r = 0; r < NT; ++r) {
          const uint16_t* hp = A::hi(cur + (16 * r + m) * RS) + g * KPL + 8 * c;
          const bf16x8 bh = *reinterpret_cast<const bf16x8*>(hp);
          const bf16x8 bl = *reinterpret_cast<const bf16x8*>(hp + CHI);
#pragma unroll
          for (int q = 0; q < MT; ++q) {
            acc[r][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Am[q], bh, acc[r][q], 0, 0, 0);
            acc[r][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Am[q], bl, acc[r][q], 0, 0, 0);
          }
        }
      }
      // per-row exponents on renormalisation steps, from a second read of
      // the rows' hi parts exactly as in pass_body (a running maximum carried
      // over the K chunks instead gave wrong values in row tiles after the
      // first; its cause was not identified, so that form is not used)
      int e[NT];
      int oe = 0;
#pragma unroll
      for (int r = 0; r < NT; ++r) {
        e[r] = 0;
        if constexpr (RN) {
          DBF16::BOp<KPL> bo;
          A::template load_b<KPL>(cur + (16 * r + m) * RS, g, bo);
          e[r] = A::template row_exp<KPL>(bo);
        }
      }
      if (RN && ot >= 0) {  // the exponent of the odd row's input row
        DBF16::BOp<KPL> bo;
        A::template load_b<KPL>(orow, g, bo);
        oe = A::template row_exp<KPL>(bo);
      }
      // exponents are read and written by wave 0 alone (program order); rows
      // are read by every wave, so in place they wait for the barrier
      int eold[NT];
      int eoin = 0;
      if (wv == 0) {
#pragma unroll
        for (int r = 0; r < NT; ++r) eold[r] = exc[16 * r + m];
        if (oin >= 0) eoin = exc[oin];
      }
      if (INPL) lds_barrier();
#pragma unroll
      for (int r = 0; r < NT; ++r) {
        const float sc = __builtin_amdgcn_ldexpf(1.f, -e[r]);  // exact power of two
#pragma unroll
        for (int q = 0; q < MT; ++q) {
          f4 v = acc[r][q];
          if constexpr (RN) {  // the scale is 1 on other steps
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] *= sc;
          }
          A::store4(nxt + (16 * r + m) * RS, 16 * (wv * MT + q) + 4 * g, v);
        }
        if (wv == 0 && g == 0) exn[16 * r + m] = eold[r] + e[r] + cexp;
      }
      if (oin >= 0) {  // lanes of column oin % 16 hold the odd row's outputs
        if (m == (oin & 15)) {
          const float sc = __builtin_amdgcn_ldexpf(1.f, -oe);
#pragma unroll
          for (int q = 0; q < MT; ++q) {
            f4 v = oacc[q];
            if constexpr (RN) {
#pragma unroll
              for (int i = 0; i < 4; ++i) v[i] *= sc;
            }
            A::store4(nxt + oout * RS, 16 * (wv * MT + q) + 4 * g, v);
          }
        }
        if (wv == 0 && lane == (oin & 15)) exn[oout] = eoin + oe + cexp;
      }
    };
    // dispatched on the tile count and, as a second template parameter, on
    // whether the step renormalises (the other steps then carry no scaling)
    auto dispatch = [&](auto rnc) {
      switch (ntile) {
#define PASS_W_CASE(x)                                                     \
  case x:                                                                 \
    if constexpr (x <= NTM) step(std::integral_constant<int, x>{}, rnc);   \
    break;
        PASS_W_CASE(1) PASS_W_CASE(2) PASS_W_CASE(3) PASS_W_CASE(4) PASS_W_CASE(5)
        PASS_W_CASE(6) PASS_W_CASE(7) PASS_W_CASE(8) PASS_W_CASE(9)
#undef PASS_W_CASE
        default: break;  // the host keeps every group within NTM tiles
      }
    };
    if (rn) dispatch(std::true_type{});
    else dispatch(std::false_type{});
    lds_barrier();
    if (!INPL) {
      float* tp = cur; cur = nxt; nxt = tp;
      int* te = exc; exc = exn; exn = te;
    }
  }
  __syncthreads();

  if (bx < a.W) {
    float* ov = a.out_vec + (((size_t)ty * a.W + w) * nslot) * CHI;
    for (int i = threadIdx.x; i < nslot * CHI; i += 256) ov[i] = A::get(cur + (i / CHI) * RS, i % CHI);
    int32_t* oe_out = a.out_exp + ((size_t)ty * a.W + w) * nslot;
    for (int i = threadIdx.x; i < nslot; i += 256) oe_out[i] = exc[i];
  }
}

template <class D, int CHI>
__device__ __forceinline__ void pass_body(const PassArgs& a, int bx, int ty) {
  if constexpr (pass_wide_form<D, CHI>()) {
    pass_body_wide<D, CHI>(a, bx, ty);
    return;
  }
  using E = typename D::elem;
  using G = Geo<CHI>;
  constexpr int WPW = G::WPW, MT = G::MT, KPL = G::KPL, RS = G::RS;
  constexpr int WPB = 4 / WPW;
  extern __shared__ __align__(16) float lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ws = wave / WPW, wv = wave % WPW;
  const int g = lane >> 4, m = lane & 15;
  const int w_raw = bx * WPB + ws;
  const int w = w_raw < a.W ? w_raw : a.W - 1;
  const int nslot = a.nslot;
  const int bufsz = nslot * RS;
  float* cur = lds + ws * (2 * bufsz);
  float* nxt = cur + bufsz;
  int* exc = reinterpret_cast<int*>(lds + WPB * 2 * bufsz) + ws * (2 * nslot);
  int* exn = exc + nslot;
  uint64_t* spw = reinterpret_cast<uint64_t*>(lds + WPB * 2 * bufsz + WPB * 2 * nslot) + ws * a.nw;

  const int tid_w = wv * 64 + lane;
  constexpr int NT_W = WPW * 64;
  for (int i = tid_w; i < 2 * bufsz; i += NT_W) cur[i] = 0.f;
  for (int i = tid_w; i < 2 * nslot; i += NT_W) exc[i] = 0;
  for (int i = tid_w; i < a.nw; i += NT_W) spw[i] = a.spins[(size_t)w * a.nw + i];
  __syncthreads();
  using A = Act<D, CHI>;
  if (tid_w == 0) A::set_unit(cur);  // boundary vector e_0 in the base slot
  __syncthreads();

  const int term = ty / a.ng, grp = ty % a.ng;
  const E* cores = static_cast<const E*>(a.cores) + (size_t)term * a.L * 2 * CHI * CHI;
  const int* cexp_p = a.core_exp ? a.core_exp + (size_t)term * a.L : nullptr;
  const int2 gs = a.gsteps[grp];
  const int4* sched = a.sched + gs.x;

  // Work items = (schedule step, group of MTI output tiles of this wave).
  // When the fragments of all MT tiles fit in registers (MTI = MT) a row
  // tile's activations are read once per step and used for every tile;
  // otherwise (bond 256) once per half of the tiles.  The core fragments of item i+1
  // are loaded while item i computes.  Rows are stored in the matrix-op
  // form (Act), and renormalisation scales the products, not the inputs.
  // (FP8 fragments are sized as BF16 ones here: the codes are decoded to
  // BF16 operands next to the matrix ops, which needs the room)
  constexpr int FRAG_DW = MT * 2 * KPL * (sizeof(E) < 2 ? 2 : (int)sizeof(E)) / 4;
  constexpr int MTI = FRAG_DW <= 128 ? MT : (MT % 2 == 0 && FRAG_DW <= 256 ? MT / 2 : 1);
  constexpr int NIS = MT / MTI;  // items per step
  constexpr bool ODD_MFMA = !D::kF32;
  struct Frags { E m[MTI][KPL]; E o[MTI][KPL]; };
  // FP8 fragments stay codes while their loads are in flight and are decoded
  // to BF16 once per item, since every row tile of the step uses them; the
  // matrix ops then run as for BF16 cores
  constexpr bool kDec = std::is_same<D, DFP8>::value;
  using DR = typename std::conditional<kDec, DBF16, D>::type;
  using ER = typename DR::elem;
  const int n_items = gs.y * NIS;
  // The other slice is read only on steps with an odd row (one step in ng
  // when the spins are dealt over ng groups); elsewhere F.o keeps whatever
  // it held and is not used.
  auto load = [&](Frags& F, int item) {
    const int s = item / NIS, ig = item % NIS;
    const int4 st = sched[s];
    const int bit = spin_bit(spw, st.y);
#pragma unroll
    for (int q = 0; q < MTI; ++q) {
      const size_t tile = (size_t)(wv * MT + ig * MTI + q) * 64 * KPL;
      load_frag<KPL>(F.m[q], cores + ((size_t)st.x * 2 + bit) * (CHI * CHI) + tile, lane);
    }
    if (st.w >= 0) {
#pragma unroll
      for (int q = 0; q < MTI; ++q) {
        const size_t tile = (size_t)(wv * MT + ig * MTI + q) * 64 * KPL;
        load_frag<KPL>(F.o[q], cores + ((size_t)st.x * 2 + (bit ^ 1)) * (CHI * CHI) + tile, lane);
      }
    }
  };
  auto compute = [&](const Frags& F, int item) {
    const int s = item / NIS, ig = item % NIS;
    const int4 st = sched[s];
    const int k = st.x, nact = st.z, odd = st.w;
    // the other slice only serves the odd row, which most steps of a row
    // group do not have: its codes are decoded only when it does
    const int oin = odd >= 0 ? (odd & 0xffff) : -1, oout = odd >> 16;
    ER Fm[MTI][KPL], Fo[MTI][KPL];
    if constexpr (kDec) {
#pragma unroll
      for (int q = 0; q < MTI; ++q) D::template decode<KPL>(F.m[q], Fm[q]);
      if (oin >= 0) {
#pragma unroll
        for (int q = 0; q < MTI; ++q) D::template decode<KPL>(F.o[q], Fo[q]);
      }
    }
    auto fm = [&](int q) -> const ER(&)[KPL] {
      if constexpr (kDec) return Fm[q];
      else return F.m[q];
    };
    auto fo = [&](int q) -> const ER(&)[KPL] {
      if constexpr (kDec) return Fo[q];
      else return F.o[q];
    };
    const int cexp = cexp_p ? cexp_p[k] : 0;
    const int ntile = (nact + 15) >> 4;
    // rows are renormalised every kRenormEvery steps: between two, a row
    // grows by at most a factor chi per step (core entries below 1)
    const bool rn = (s % kRenormEvery) == 0;
    // With BF16 cores the odd row rides on the matrix cores too: when the
    // row tile holding its input comes by, the other slice is applied to the
    // same B operand and the column of that row kept (stored after the loop,
    // since the main loop may also write its output slot).  FP32 matrix ops
    // are 8x slower, so there it stays a vector-ALU dot product.
    f4 oacc[MTI];
    int oe = 0;
    for (int r = 0; r < ntile; ++r) {
      const int row = 16 * r + m;
      typename D::template BOp<KPL> bo;
      A::template load_b<KPL>(cur + row * RS, g, bo);
      const int e = rn ? A::template row_exp<KPL>(bo) : 0;
      const float sc = __builtin_amdgcn_ldexpf(1.f, -e);  // exact power of two
      if (ig == 0 && wv == 0 && g == 0) exn[row] = exc[row] + e + cexp;
#pragma unroll
      for (int q = 0; q < MTI; ++q) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = DR::template mma<KPL>(fm(q), bo, acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] *= sc;
        A::store4(nxt + row * RS, 16 * (wv * MT + ig * MTI + q) + 4 * g, acc);
      }
      if (ODD_MFMA && r == (oin >> 4)) {
        oe = e;
#pragma unroll
        for (int q = 0; q < MTI; ++q) {
          f4 acc = {0.f, 0.f, 0.f, 0.f};
          acc = DR::template mma<KPL>(fo(q), bo, acc);
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[i] *= sc;
          oacc[q] = acc;
        }
      }
    }
    if (ODD_MFMA && oin >= 0) {  // lanes of column oin % 16 hold 4 output features each
      if (m == (oin & 15)) {
#pragma unroll
        for (int q = 0; q < MTI; ++q) A::store4(nxt + oout * RS, 16 * (wv * MT + ig * MTI + q) + 4 * g, oacc[q]);
      }
      if (ig == 0 && wv == 0 && lane == (oin & 15)) exn[oout] = exc[oin] + oe + cexp;
    }
    if (!ODD_MFMA && oin >= 0) {  // FP32: the odd row as a vector-ALU dot product per output
      float v[KPL];
      A::template load_f32<KPL>(cur + oin * RS, g, v);
      int e = 0;
      if (rn) {
        float mx = 0.f;
#pragma unroll
        for (int c = 0; c < KPL; ++c) mx = fmaxf(mx, fabsf(v[c]));
        mx = group_max(mx);
        e = (mx > 0.f) ? __builtin_amdgcn_frexp_expf(mx) : 0;
      }
#pragma unroll
      for (int q = 0; q < MTI; ++q) {
        float p = 0.f;
#pragma unroll
        for (int c = 0; c < KPL; ++c) p = fmaf(DR::to_f32(F.o[q][c]), v[c], p);
        p += __shfl_xor(p, 16);
        p += __shfl_xor(p, 32);
        if (g == 0) A::store1(nxt + oout * RS, 16 * (wv * MT + ig * MTI + q) + m, __builtin_amdgcn_ldexpf(p, -e));
      }
      if (ig == 0 && wv == 0 && lane == 0) exn[oout] = exc[oin] + e + cexp;
    }
    if (ig == NIS - 1) {
      lds_barrier();
      float* tp = cur; cur = nxt; nxt = tp;
      int* te = exc; exc = exn; exn = te;
    }
  };
  // A ring of PFP fragment sets: loads run PFP - 1 items ahead of the
  // matrix ops, issued on every path (clamped to the last item) so that the
  // wait before the matrix ops never covers an item still being prefetched.
  // Two sets everywhere: a third (the FP8 sets are half the registers of
  // BF16 ones) measured slower at bond 256, and at bond 128 it costs the
  // kernel its second wave per SIMD.
  constexpr int PFP = (kDec && CHI == 256) ? PASS_PF_FP8 : 2;
  Frags FR[PFP];
  if (n_items > 0) {
#pragma unroll
    for (int q = 0; q < PFP - 1; ++q) load(FR[q], min(q, n_items - 1));
    for (int i = 0; i < n_items; i += PFP) {
#pragma unroll
      for (int r = 0; r < PFP; ++r) {
        if (i + r >= n_items) break;
        load(FR[(r + PFP - 1) % PFP], min(i + r + PFP - 1, n_items - 1));
        compute(FR[r], i + r);
      }
    }
  }
  __syncthreads();

  if (w_raw < a.W) {
    float* ov = a.out_vec + (((size_t)ty * a.W + w) * nslot) * CHI;
    for (int i = tid_w; i < nslot * CHI; i += NT_W) ov[i] = A::get(cur + (i / CHI) * RS, i % CHI);
    int32_t* oe = a.out_exp + ((size_t)ty * a.W + w) * nslot;
    for (int i = tid_w; i < nslot; i += NT_W) oe[i] = exc[i];
  }
}

template <class D, int CHI>
__global__ void __launch_bounds__(256, (pass_min_blocks<D, CHI>())) pass_kernel(PassArgs a) {
  pass_body<D, CHI>(a, blockIdx.x, blockIdx.y);  // y = term * ng + group
}

// ============================================================================
// combine kernel (one wave per walker)
// ============================================================================
struct CombineArgs {
  const float* u; const int32_t* ue;  // forward  [T][ng][W][nsf][chi], [T][ng][W][nsf]
  const float* v; const int32_t* ve;  // backward [T][ng][W][nsb][chi], [T][ng][W][nsb]
  int nsf, nsb, chi, T, W, N, nw, ng;
  const int32_t* fslot;               // [N] forward slot of spin j in its group (0 = base)
  const int32_t* bslot;               // [N] backward slot of spin j in its group (0 = base)
  const int32_t* grp;                 // [N] row group of spin j
  const double* coeffs;               // [T]
  const uint64_t* spins;
  const int2* bonds; int nbonds; double J, h;
  double* logabs; int8_t* sign; double* logratio; int8_t* rsign; double* eloc; int32_t* status;
};

// value = mant * 2^ex with |mant| in [0.5, 1) (mant = 0 for zero) of the
// combined amplitude whose forward row is slot fs and backward row slot bs
// of row group gi.  Sixteen lanes (c16 = lane % 16) share one dot product:
// each reads every 16th float4 of the two rows (coalesced 256-byte runs per
// row), FP64 partial sums meet by butterfly; all sixteen lanes return it.
__device__ inline void combined_value(const CombineArgs& a, int w, int gi, int fs, int bs, int c16,
                                      double& mant, int& ex) {
  double ms[kMaxTerms];
  int es[kMaxTerms];
  int emax = INT_MIN;
  for (int t = 0; t < a.T; ++t) {
    const size_t ty = (size_t)t * a.ng + gi;
    const float* pu = a.u + ((ty * a.W + w) * a.nsf + fs) * a.chi;
    const float* pv = a.v + ((ty * a.W + w) * a.nsb + bs) * a.chi;
    double d = 0.0;
    for (int f = 4 * c16; f < a.chi; f += 64) {
      const float4 x = *reinterpret_cast<const float4*>(pu + f);
      const float4 y = *reinterpret_cast<const float4*>(pv + f);
      d = fma((double)x.x, (double)y.x, d);
      d = fma((double)x.y, (double)y.y, d);
      d = fma((double)x.z, (double)y.z, d);
      d = fma((double)x.w, (double)y.w, d);
    }
    d += __shfl_xor(d, 8);
    d += __shfl_xor(d, 4);
    d += __shfl_xor(d, 2);
    d += __shfl_xor(d, 1);
    int ed = 0;
    const double md = frexp(d, &ed);
    ms[t] = a.coeffs[t] * md;
    es[t] = a.ue[(ty * a.W + w) * a.nsf + fs] + a.ve[(ty * a.W + w) * a.nsb + bs] + ed;
    if (ms[t] != 0.0 && es[t] > emax) emax = es[t];
  }
  if (emax == INT_MIN) { mant = 0.0; ex = 0; return; }
  double S = 0.0;
  for (int t = 0; t < a.T; ++t)
    if (ms[t] != 0.0) S += ldexp(ms[t], es[t] - emax);
  int eS = 0;
  mant = frexp(S, &eS);
  ex = emax + eS;
}

__device__ inline double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// One wave per walker; the wave's four 16-lane groups take four spins at a
// time.  Writes log|psi|, sign, status, every log|r_j| and sign, and E_loc.
__device__ __forceinline__ void combine_body(const CombineArgs& a, int bx) {
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, c16 = lane & 15;
  const int w = bx * 4 + (threadIdx.x >> 6);
  if (w >= a.W) return;
  const double LN2 = 0.69314718055994530942;
  double m0; int e0;
  combined_value(a, w, 0, 0, 0, c16, m0, e0);
  const bool ok = (m0 != 0.0) && isfinite(m0);
  const double lab0 = ok ? log(fabs(m0)) + e0 * LN2 : NAN;
  if (lane == 0) {
    if (a.logabs) a.logabs[w] = lab0;
    if (a.sign) a.sign[w] = ok ? (m0 > 0 ? 1 : -1) : 0;
    if (a.status) a.status[w] = ok ? 0 : -5;
  }
  double rsum = 0.0;
  for (int j0 = 0; j0 < a.N; j0 += 4) {
    const bool valid = j0 + q < a.N;
    const int j = valid ? j0 + q : a.N - 1;  // every group takes part in its butterfly
    const int fs = a.fslot[j], bs = a.bslot[j];
    double lr = NAN, r = NAN;
    int8_t sg = 0;
    if (ok) {
      if (fs == 0 && bs == 0) {  // spin read by no position: r_j = 1 exactly
        lr = 0.0; sg = 1; r = 1.0;
      } else {
        double mj; int ej;
        combined_value(a, w, a.grp[j], fs, bs, c16, mj, ej);
        if (mj == 0.0) { lr = -INFINITY; sg = 1; r = 0.0; }
        else {
          // the ratio from the mantissa quotient and the exponent difference
          // (no logarithms unless log-ratios are asked for)
          const double qm = fabs(mj) / fabs(m0);
          sg = ((mj > 0) == (m0 > 0)) ? 1 : -1;
          r = sg * ldexp(qm, ej - e0);
          if (a.logratio) lr = log(qm) + (double)(ej - e0) * LN2;
        }
      }
    }
    if (valid && c16 == 0) {
      if (a.logratio) a.logratio[(size_t)w * a.N + j] = lr;
      if (a.rsign) a.rsign[(size_t)w * a.N + j] = sg;
      rsum += ok ? r : 0.0;
    }
  }
  if (a.eloc) {
    const uint64_t* sw = a.spins + (size_t)w * a.nw;
    double diag = 0.0;
    for (int b = lane; b < a.nbonds; b += 64) {
      const int2 bd = a.bonds[b];
      diag += (spin_bit(sw, bd.x) ^ spin_bit(sw, bd.y)) ? -1.0 : 1.0;
    }
    diag = wave_sum(diag);
    rsum = wave_sum(rsum);
    if (lane == 0) a.eloc[w] = ok ? a.J * diag - a.h * rsum : NAN;
  }
}

__global__ void __launch_bounds__(256) combine_kernel(CombineArgs a) { combine_body(a, blockIdx.x); }

// ============================================================================
// chain kernel: 16 walkers per block, amplitudes and Metropolis sweeps
// ============================================================================
struct ChainArgs {
  const void* cores;         // [T][L][2][CHI*CHI] forward fragment layout (prescaled)
  const void* cores_bwd;     // [T][L][2][CHI*CHI] backward fragment layout (prescaled)
  const int32_t* cesum;      // [T][L+1] prefix sums of the per-position scale exponents
  const int32_t* pi;         // [L]
  const uint64_t* rmask;     // [N][LW] bit k set iff position k reads spin j
  const int32_t* order;      // [N] proposal order
  const int32_t* first;      // [N] first position of spin j, -1 if none
  const double* coeffs;      // [T]
  int T, L, N, nw, LW, W;
  uint64_t* spins;
  double* logabs; int8_t* sign; uint32_t* accepts; int32_t* status;
  uint64_t seed, rstream, sweep0;
  int n_sweeps;
  int mode;                  // 0: amplitudes only, 1: sweeps
  // Column checkpoints (sweeps): the right environments of bonds
  // ck_first + i * ck_step, i < n_ck, for the current configuration, with a
  // per-walker validity mask (0: none); kept in LDS, or in global memory
  // (ckg) with the sequential layout.
  int n_ck, ck_first, ck_step;
  // With the term-by-term ("sequential") layout the checkpoint vectors live
  // in global memory: [block][saved, candidate][n_ck][T][16 cg walkers][bond + 4],
  // room for ck_cap checkpoints
  float* ckg;
  int ck_cap;
};

// Layout of one block's walkers' state in LDS (offsets in bytes), for
// nb = 16 * cg walkers.  Per term: the prefix row P, the first-step products
// U and F, row ping-pong X/Y and column ping-pong CX/CY (7 buffers), all
// terms advancing together when that fits; otherwise ("sequential") each
// term keeps only its prefix and the terms share F, X, Y, CX, CY, one term
// at a time, the prefix being advanced after the decision.  Vectors are
// stored buffer-major ([buffer][term]); with all terms together nck column
// checkpoints per term and as many candidates follow as buffers 7 ...
// 6 + 2 nck (with the sequential layout those vectors are in global memory),
// their exponents after the spins, and last the replica bitmasks of the
// n_spins spins when they fit (else they are read from global memory).
struct ChainLayout {
  int nb, rows, exps, vals, pm, sp, ckexp, rm, total;
  bool seq, rml;
  __host__ __device__ ChainLayout(int chi, int T, int LW, int nw, int cg, int nck, int n_spins) {
    nb = 16 * cg;
    const int bufb = nb * (chi + 4) * 4;
    const int tail = 4 * T * nb * 4 + T * nb * 12 + 8 + nb * LW * 8 + nb * nw * 8;
    seq = (T * 7 * bufb + tail) > 160 * 1024;   // (seq: checkpoint vectors in global memory)
    rows = 0;                                                 // float vectors
    exps = rows + (seq ? T + 5 : (7 + 2 * nck) * T) * bufb;  // int [4][T][nb]: prefix, first step, row, column
    vals = exps + 4 * T * nb * 4;                  // double [T][nb] end values, int [T][nb] exponents
    pm = vals + T * nb * 12;
    pm = (pm + 7) & ~7;
    sp = pm + nb * LW * 8;                         // uint64 [nb][LW] position bits; [nb][nw] spins
    ckexp = sp + nb * nw * 8;                      // int [2][nck][T][nb] checkpoint exponents
    total = ckexp + 2 * nck * T * nb * 4;
    rm = (total + 7) & ~7;                         // uint64 [n_spins][LW] replica bitmasks
    rml = rm + n_spins * LW * 8 <= 160 * 1024;
    if (rml) total = rm + n_spins * LW * 8;
  }
};

// Waves per side of the chain kernel: two sides of up to four waves, except
// that wide bonds keep one wave per SIMD (their fragments need the whole
// register file) with two waves per side.
template <int CHI, class D = DBF16>
struct ChainGeo {
  // waves per side: FP8 fragments are half the registers of BF16 ones, but
  // four waves per side at bond 256 (two per SIMD) still spill, so
  // CHAIN_SW_FP8_256 keeps two
  static constexpr int SW = (CHI == 256 && std::is_same<D, DFP8>::value) ? CHAIN_SW_FP8_256
                            : CHI >= 128 ? 2 : Geo<CHI>::WPW;
  static constexpr int MT = CHI / (16 * SW);                   // output tiles per wave
  static constexpr int NT = 2 * SW * 64;                       // threads per block
  // fragment sets in the prefetch ring (see chain_body)
  template <class E>
  static constexpr int PF = ((CHI == 128 && sizeof(E) == 2) || (CHI == 128 && sizeof(E) == 1)) ? 4
                            : (CHI == 256 && sizeof(E) == 1) ? CHAIN_PF_FP8_256 : 2;
};

// Block of 2 * SW waves for 16 * CG walkers: CG groups of 16 matrix-core
// columns that share every core fragment a wave loads (more walkers per
// fragment when there are enough walkers to fill the GPU).  Every amplitude
// is contracted from both ends at once: the first SW waves carry row vectors
// from the left (forward fragment layout), the other SW waves column vectors
// from the right boundary (backward layout); the two meet half way and are
// joined by an FP64 dot product.  The number of dependent steps per
// amplitude is halved and each SIMD runs two independent chains.  CKP
// compiles the column checkpoints in: kept in LDS at bonds up to 64 (wider
// bonds leave LDS for too few of them), and with CKG in global memory for
// the term-sequential layout of FP8 cores at bond 256 (other bond-128 and
// bond-256 kernels are register-bound and stay without them).
template <class D, int CHI, int CG, bool CKP = false, bool CKG = false>
__device__ __forceinline__ void chain_body(const ChainArgs& a, int bx, uint64_t sweep0) {
  using E = typename D::elem;
  using G = Geo<CHI>;
  constexpr int RS = G::RS, KPL = G::KPL;
  // Prefetch ring of fragment sets: 4 for BF16 fragments at bond 128 (10x10
  // sweep 37.4 -> 30.9 ms), 2 elsewhere (deeper rings slowed the bond-64
  // sweep; FP32 at 128 would spill and at 256 the fragments would not fit
  // the register file).
  constexpr int MT = ChainGeo<CHI, D>::MT, SW = ChainGeo<CHI, D>::SW, PF = ChainGeo<CHI, D>::template PF<E>;
  constexpr int NB = 16 * CG;
  constexpr int BUF = NB * RS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int side = wave / SW;    // 0: rows from the left, 1: columns from the right
  const int wv = wave % SW;      // wave within its side
  const int g = lane >> 4, m = lane & 15;
  const int nthr = blockDim.x, nwave = nthr >> 6;
  const int T = a.T, L = a.L, LW = a.LW, nw = a.nw;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const ChainLayout lay(CHI, T, LW, nw, CG, a.n_ck, a.N);
  float* rows = reinterpret_cast<float*>(lds_raw + lay.rows);
  int* Ep = reinterpret_cast<int*>(lds_raw + lay.exps);   // [T][NB] prefix
  int* Ef = Ep + T * NB;                                   // [T][NB] after the first step
  int* Er = Ef + T * NB;                                   // [T][NB] running row
  int* Ec = Er + T * NB;                                   // [T][NB] running column
  double* fval = reinterpret_cast<double*>(lds_raw + lay.vals);  // [T][NB] amplitude mantissas
  int* fexp = reinterpret_cast<int*>(fval + T * NB);             // [T][NB] their exponents
  uint64_t* pm = reinterpret_cast<uint64_t*>(lds_raw + lay.pm);
  uint64_t* sp = reinterpret_cast<uint64_t*>(lds_raw + lay.sp);
  const bool seq = lay.seq;
  const int nbuf = seq ? T + 5 : 7 * T;
  const int NCK = CKP ? a.n_ck : 0;
  int* cke = reinterpret_cast<int*>(lds_raw + lay.ckexp);

  // Buffer ids: the seven vectors of a term, then CK + i for the saved
  // column of checkpoint i and CD + i for its candidate.
  enum { P = 0, U = 1, F = 2, X = 3, Y = 4, CX = 5, CY = 6, CK = 7 };
  const int CD = CK + NCK;
  auto buf = [&](int t, int b) {
    if (!seq) return rows + (b * T + t) * BUF;
    return b == P ? rows + t * BUF : rows + (T + b - F) * BUF;  // U is not used then
  };
  // CKG (sequential layout only): the checkpoint vectors are in global
  // memory, addressed by gbuf and accessed non-temporally (they must not
  // push the core fragments out of L2); a segment starting from one first copies it
  // into the spare column buffer, so that every vector access of the steps
  // stays an LDS access.
  float* ckg = (CKG && NCK > 0) ? a.ckg + (size_t)bx * 2 * NCK * T * BUF : nullptr;
  auto gbuf = [&](int t, int b) { return ckg + ((size_t)(b - CK) * T + t) * BUF; };
  auto ckexp = [&](int b, int t, int wn) -> int& { return cke[((b - CK) * T + t) * NB + wn]; };
  // index of the first checkpoint whose bond is >= b (NCK if none)
  auto ck_ceil = [&](int b) {
    const int d = b - a.ck_first;
    return d <= 0 ? 0 : min(NCK, (d + a.ck_step - 1) / a.ck_step);
  };
  // bits [lo, hi) of a checkpoint mask
  auto ck_bits = [](int lo, int hi) -> uint32_t {
    return hi > lo ? ((1u << hi) - 1u) & ~((1u << lo) - 1u) : 0u;
  };

  const int w0 = bx * NB;
  bool live[CG];
#pragma unroll
  for (int cg = 0; cg < CG; ++cg) live[cg] = (w0 + 16 * cg + m) < a.W;
  for (int i = threadIdx.x; i < nbuf * BUF; i += nthr) rows[i] = 0.f;
  for (int i = threadIdx.x; i < 4 * T * NB; i += nthr) Ep[i] = 0;
  for (int i = threadIdx.x; i < NB * nw; i += nthr) {
    const int n = i / nw, wd = i % nw;
    sp[i] = (w0 + n < a.W) ? a.spins[(size_t)(w0 + n) * nw + wd] : 0ull;
  }
  // replica bitmask word wd of spin j (from LDS when the masks fit there)
  uint64_t* rml = reinterpret_cast<uint64_t*>(lds_raw + lay.rm);
  if (lay.rml)
    for (int i = threadIdx.x; i < a.N * LW; i += nthr) rml[i] = a.rmask[i];
  auto rword = [&](int j, int wd) -> uint64_t {
    uint64_t x;
    if (lay.rml) x = rml[j * LW + wd];
    else x = a.rmask[(size_t)j * LW + wd];
    return x;
  };
  __syncthreads();
  for (int i = threadIdx.x; i < NB * LW; i += nthr) {
    const int n = i / LW, wd = i % LW;
    uint64_t word = 0;
    for (int b = 0; b < 64 && 64 * wd + b < L; ++b) {
      const int q = a.pi[64 * wd + b];
      word |= (uint64_t)spin_bit(sp + n * nw, q) << b;
    }
    pm[i] = word;
  }

  const E* cores = static_cast<const E*>(side == 0 ? a.cores : a.cores_bwd);
  struct Frags { E f0[KPL]; E f1[KPL]; };
  // vectors are kept in LDS in the form the matrix ops take (Act: FP32, or
  // the hi and lo BF16 parts), split once by the wave that writes them;
  // renormalisation scales the products, not the stored inputs
  using A = Act<D, CHI>;
  typename D::template BOp<KPL> bo[CG];
  float psc[CG];

  // Results of the last segment: rb holds the rows, cb the columns (-1: the
  // right boundary vector itself).  Every wave knows both.
  int rb = P, cb = -1;

  // For terms [t0, t0+tn) with spin jflip flipped (-1: none): advance the
  // row vectors from P through positions [k0, k1) and, at the same time,
  // column vectors from bond ks (the right boundary if ks = L, else the
  // saved column of that checkpoint) through positions ks-1 down to kc.
  // Columns reaching a checkpoint bond are kept: as its saved column when
  // the bond lies past lj, the last position of the flipped spin (they are
  // then the current configuration's), else as its candidate.
  // Work items of a wave are (step, term, output tile) in that order; the
  // two core fragments of the next item are loaded while the current one
  // computes, and each serves all CG column groups.  Each joint step ends
  // with one block barrier (the side with fewer steps still takes part).
  // With `split` the first row step stores the walker's own slice product in
  // F and the other slice's in U.  Vectors are renormalised every
  // kRenormEvery steps; the exponent sums live in Er and Ec.
  auto segment = [&](int k0, int k1, int kc, int ks, int lj, int jflip, bool split, int t0, int tn) {
    const int nr = k1 > k0 ? k1 - k0 : 0, nc = ks - kc;
    const int cks = (CKP && ks < L) ? CK + (ks - a.ck_first) / a.ck_step : -1;
    // the buffer the columns start from: the checkpoint itself, or with
    // CKG its copy in the spare column buffer CY (the steps write CX first)
    int ck_src = cks;
    if constexpr (CKG) {
      if (cks >= 0) {
        for (int i = threadIdx.x; i < tn * (BUF / 4); i += nthr) {
          const int t = t0 + i / (BUF / 4), r = i % (BUF / 4);
          reinterpret_cast<f4*>(buf(t, CY))[r] = __builtin_nontemporal_load(reinterpret_cast<const f4*>(gbuf(t, cks)) + r);
        }
        lds_barrier();
        ck_src = CY;
      }
    }
    if (nr == 0) rb = P;
    else if (split) rb = nr == 1 ? F : (((nr - 1) & 1) ? X : Y);
    else rb = (nr & 1) ? X : Y;
    cb = nc == 0 ? ck_src : ((nc & 1) ? CX : CY);
    const int S = nr > nc ? nr : nc;
    const int n = side == 0 ? nr : nc;
    if (CKP && side == 1 && n == 0 && cks >= 0 && wv == 0 && g == 0)
      for (int t = t0; t < t0 + tn; ++t)
#pragma unroll
        for (int cg = 0; cg < CG; ++cg) Ec[t * NB + 16 * cg + m] = ckexp(cks, t, 16 * cg + m);
    if (n > 0) {

      int cur = side == 0 ? P : ck_src;
      int out = side == 0 ? (split ? F : X) : CX;
      const int tend = t0 + tn;
      int i = 0, t = t0, mt = 0;
      // the next checkpoint the columns reach (bond ckb, index cki; -1: none)
      int cki = -1, ckb = -1;
      if (CKP && side == 1 && NCK > 0 && ks - 1 >= a.ck_first) {
        cki = min(NCK - 1, (ks - 1 - a.ck_first) / a.ck_step);
        ckb = a.ck_first + cki * a.ck_step;
      }
      int bit[CG];
      uint64_t word[CG];
#pragma unroll
      for (int cg = 0; cg < CG; ++cg) { bit[cg] = 0; word[cg] = 0; }
      auto pos_of = [&](int ii) { return side == 0 ? k0 + ii : ks - 1 - ii; };
      auto load = [&](Frags& Fr, int ii, int tt, int mm) {
        const int kk = pos_of(ii < n ? ii : n - 1);
        const E* base = cores + (((size_t)tt * L + kk) * 2) * (CHI * CHI) +
                        (size_t)(wv * MT + mm) * 64 * KPL;
        load_frag<KPL>(Fr.f0, base, lane);
        load_frag<KPL>(Fr.f1, base + CHI * CHI, lane);
      };
      auto step = [&](const Frags& Fr) {
        const int k = pos_of(i);
        if (t == t0 && mt == 0) {
          const bool fresh = i == 0 || (k & 63) == (side == 0 ? 0 : 63);
#pragma unroll
          for (int cg = 0; cg < CG; ++cg) {
            if (fresh) word[cg] = pm[(16 * cg + m) * LW + (k >> 6)] ^ (jflip >= 0 ? rword(jflip, k >> 6) : 0ull);
            bit[cg] = (int)((word[cg] >> (k & 63)) & 1ull);
          }
        }
        if (mt == 0) {
#pragma unroll
          for (int cg = 0; cg < CG; ++cg) {
            const int wn = 16 * cg + m;
            psc[cg] = 1.f;
            if (cur < 0) {  // the right boundary vector e_0
              float v[KPL];
#pragma unroll
              for (int e = 0; e < KPL; ++e) v[e] = (g == 0 && e == 0) ? 1.f : 0.f;
              D::template prep<KPL>(v, bo[cg]);
              if (wv == 0 && g == 0) Ec[t * NB + wn] = 0;
            } else {
              // FP32 rows are renormalised in place as read; BF16 rows scale
              // the products instead (their stored split stays as written)
              float v[KPL];
              if constexpr (D::kF32) lds_read<KPL>(v, buf(t, cur) + wn * RS + g * KPL);
              else A::template load_b<KPL>(buf(t, cur) + wn * RS, g, bo[cg]);
              if (i % kRenormEvery == 0) {
                int e;
                if constexpr (D::kF32) {
                  e = renorm_row<KPL>(v);
                } else {
                  e = A::template row_exp<KPL>(bo[cg]);
                  psc[cg] = __builtin_amdgcn_ldexpf(1.f, -e);  // exact power of two
                }
                if (wv == 0 && g == 0) {
                  if (side == 1) {
                    Ec[t * NB + wn] = ((CKP && i == 0) ? ckexp(cks, t, wn) : Ec[t * NB + wn]) + e;
                  } else if (split && i == 0) {
                    const int ne = Ep[t * NB + wn] + e;
                    Ef[t * NB + wn] = ne;
                    Er[t * NB + wn] = ne;
                  } else {
                    Er[t * NB + wn] = (i == 0 ? Ep[t * NB + wn] : Er[t * NB + wn]) + e;
                  }
                }
              }
              if constexpr (D::kF32) D::template prep<KPL>(v, bo[cg]);
            }
          }
        }
        const int tt = wv * MT + mt;
        f4 c0[CG], c1[CG];
#pragma unroll
        for (int cg = 0; cg < CG; ++cg) {
          c0[cg] = f4{0.f, 0.f, 0.f, 0.f};
          c1[cg] = f4{0.f, 0.f, 0.f, 0.f};
          D::template mma2<KPL>(Fr.f0, Fr.f1, bo[cg], c0[cg], c1[cg]);
        }
#pragma unroll
        for (int cg = 0; cg < CG; ++cg) {
          const int wn = 16 * cg + m;
          if constexpr (!D::kF32) {
#pragma unroll
            for (int q = 0; q < 4; ++q) { c0[cg][q] *= psc[cg]; c1[cg][q] *= psc[cg]; }
          }
          const f4 sel = bit[cg] ? c1[cg] : c0[cg];
          A::store4(buf(t, out) + wn * RS, 16 * tt + 4 * g, sel);
          if (split && side == 0 && i == 0) {
            const f4 oth = bit[cg] ? c0[cg] : c1[cg];
            A::store4(buf(t, U) + wn * RS, 16 * tt + 4 * g, oth);
          }
        }
        if (CKP && k == ckb) {  // columns only
          const int slot = k > lj ? CK + cki : CD + cki;
#pragma unroll
          for (int cg = 0; cg < CG; ++cg) {
            const int wn = 16 * cg + m;
            const f4 sel = bit[cg] ? c1[cg] : c0[cg];
            if constexpr (CKG) A::store4_nt(gbuf(t, slot) + wn * RS, 16 * tt + 4 * g, sel);
            else A::store4(buf(t, slot) + wn * RS, 16 * tt + 4 * g, sel);
            if (wv == 0 && g == 0 && mt == 0) ckexp(slot, t, wn) = Ec[t * NB + wn];
          }
        }
        if (mt == MT - 1 && t == tend - 1) {
          if (CKP && k == ckb) {
            --cki;
            ckb = cki >= 0 ? ckb - a.ck_step : -1;
          }
          lds_barrier();
          cur = out;
          out = side == 0 ? ((cur == X) ? Y : X) : ((cur == CX) ? CY : CX);
        }
        if (++mt == MT) { mt = 0; if (++t == tend) { t = t0; ++i; } }
      };
      auto next_of = [&](int& ii, int& tt, int& mm) {
        if (++mm == MT) { mm = 0; if (++tt == tend) { tt = t0; ++ii; } }
      };
      // A ring of PF fragment sets: the loads run PF - 1 items ahead of the
      // matrix ops.  They are issued on every path (past the end they
      // re-read the last position) so the number of loads in flight is the
      // same on all paths and each wait covers only the item about to be used.
      Frags FR[PF];
      int li = 0, lt = t0, lm = 0;  // load cursor
#pragma unroll
      for (int q = 0; q < PF - 1; ++q) {
        load(FR[q], li, lt, lm);
        next_of(li, lt, lm);
      }
      while (true) {
#pragma unroll
        for (int r = 0; r < PF; ++r) {
          load(FR[(r + PF - 1) % PF], li, lt, lm);
          next_of(li, lt, lm);
          step(FR[r]);
          if (i >= n) goto segment_done;
        }
      }
    segment_done:;
    }
    for (int r = n; r < S; ++r) lds_barrier();
  };

  // Join rows rb and columns cb of terms [t0, t0+tn): FP64 dot product per
  // walker (one wave per term, four lanes per walker) and its exponent.
  auto record = [&](int t0, int tn) {
    for (int t = t0 + wave; t < t0 + tn; t += nwave) {
#pragma unroll
      for (int cg = 0; cg < CG; ++cg) {
        const int wn = 16 * cg + m;
        float r[KPL];
        A::template load_f32<KPL>(buf(t, rb) + wn * RS, g, r);
        double s = 0.0;
        if (cb < 0) {
          s = (g == 0) ? (double)r[0] : 0.0;
        } else {
          float c[KPL];
          A::template load_f32<KPL>(buf(t, cb) + wn * RS, g, c);
          for (int e = 0; e < KPL; ++e) s = fma((double)r[e], (double)c[e], s);
        }
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        if (g == 0) {
          fval[t * NB + wn] = s;
          fexp[t * NB + wn] = Er[t * NB + wn] + (cb < 0 ? 0 : Ec[t * NB + wn]) +
                              a.cesum[(size_t)t * (L + 1) + L];
        }
      }
    }
    __syncthreads();
  };
  // combined amplitude of walker slot wn from the recorded values: log|psi|
  // and sign (every lane of every wave computes it for its walkers)
  auto amp = [&](int wn, double& labs, int& sg) {
    double ms[kMaxTerms];
    int es[kMaxTerms];
    int emax = INT_MIN;
    for (int t = 0; t < T; ++t) {
      int ed = 0;
      const double md = frexp(fval[t * NB + wn], &ed);
      ms[t] = a.coeffs[t] * md;
      es[t] = fexp[t * NB + wn] + ed;
      if (ms[t] != 0.0 && es[t] > emax) emax = es[t];
    }
    if (emax == INT_MIN) { labs = -INFINITY; sg = 0; return; }
    double S = 0.0;
    for (int t = 0; t < T; ++t)
      if (ms[t] != 0.0) S += ldexp(ms[t], es[t] - emax);
    int eS = 0;
    const double mS = frexp(S, &eS);
    if (mS == 0.0 || !isfinite(mS)) { labs = (mS == 0.0) ? -INFINITY : NAN; sg = 0; return; }
    labs = log(fabs(mS)) + (double)(emax + eS) * 0.69314718055994530942;
    sg = mS > 0 ? 1 : -1;
  };

  auto reset_prefix = [&]() {
    for (int i = threadIdx.x; i < T * NB * RS; i += nthr) {
      const int t = i / (NB * RS), r = i % (NB * RS);
      buf(t, P)[r] = (r % RS == 0) ? A::unit_dword() : 0.f;
    }
    for (int i = threadIdx.x; i < T * NB; i += nthr) Ep[i] = 0;
  };
  // the meeting bond of a contraction over positions [f, ks)
  auto meet = [&](int f, int ks) { return f + (ks - f + 1) / 2; };
  // bond of checkpoint i
  auto ck_bond = [&](int i) { return a.ck_first + i * a.ck_step; };

  // amplitude of the current configuration (identical in every lane of a walker)
  reset_prefix();
  __syncthreads();
  double lab[CG];
  int sgn[CG], stat[CG];
  uint32_t nacc[CG];
  const int c0 = meet(0, L);
  if (!seq) {
    segment(0, c0, c0, L, -1, -1, false, 0, T);
    record(0, T);
  } else {
    for (int t = 0; t < T; ++t) {
      segment(0, c0, c0, L, -1, -1, false, t, 1);
      record(t, 1);
    }
  }
  // checkpoints the columns passed are valid (same mask in every lane of a
  // walker, in every wave)
  uint32_t vmask[CG];
  {
    uint32_t v0 = 0;
    for (int i = 0; i < NCK; ++i)
      if (ck_bond(i) >= c0) v0 |= 1u << i;
#pragma unroll
    for (int cg = 0; cg < CG; ++cg) vmask[cg] = v0;
  }
#pragma unroll
  for (int cg = 0; cg < CG; ++cg) {
    amp(16 * cg + m, lab[cg], sgn[cg]);
    stat[cg] = (sgn[cg] != 0 && isfinite(lab[cg])) ? 0 : -5;
    nacc[cg] = 0;
  }
  __syncthreads();

  if (a.mode == 1) {
    for (int ts = 0; ts < a.n_sweeps; ++ts) {
      const uint64_t sweep = sweep0 + (uint64_t)ts;
      reset_prefix();
      __syncthreads();
      int pos = 0;
      for (int qi = 0; qi < a.N; ++qi) {
        const int j = a.order[qi];
        const int f = a.first[j];
        if (f < 0) {  // spin read by no position: ratio 1, always accepted
#pragma unroll
          for (int cg = 0; cg < CG; ++cg)
            if (live[cg] && stat[cg] == 0) {
              nacc[cg] += 1;
              if (wave == 0 && g == 0) sp[(16 * cg + m) * nw + (j >> 6)] ^= (1ull << (j & 63));
            }
          __syncthreads();
          continue;
        }
        // bring the prefix of terms [t0, t0+tn) from pos up to position kk
        auto advance_prefix = [&](int kk, int t0, int tn) {
          segment(pos, kk, L, L, -1, -1, false, t0, tn);
          for (int i = threadIdx.x; i < tn * NB * RS; i += nthr) {
            const int t = t0 + i / (NB * RS), r = i % (NB * RS);
            buf(t, P)[r] = buf(t, rb)[r];
          }
          for (int i = threadIdx.x; i < tn * NB; i += nthr) Ep[t0 * NB + i] = Er[t0 * NB + i];
          __syncthreads();
        };
        if (pos < f) {
          if (!seq) advance_prefix(f, 0, T);
          else for (int t = 0; t < T; ++t) advance_prefix(f, t, 1);
          pos = f;
        }
        // the columns start from the first checkpoint past the spin's last
        // position that every walker of the block holds valid (else from
        // the right boundary)
        int lj = -1;
        for (int wd = LW - 1; wd >= 0; --wd) {
          const uint64_t x = rword(j, wd);
          if (x) { lj = 64 * wd + 63 - __clzll((long long)x); break; }
        }
        int ks = L;
        const int il = ck_ceil(lj + 1);  // checkpoints below il lie at or before lj
        if (CKP && NCK > 0) {
          uint32_t av = ~0u;
#pragma unroll
          for (int cg = 0; cg < CG; ++cg) {
            uint32_t x = vmask[cg];
            x &= (uint32_t)__shfl_xor((int)x, 1);
            x &= (uint32_t)__shfl_xor((int)x, 2);
            x &= (uint32_t)__shfl_xor((int)x, 4);
            x &= (uint32_t)__shfl_xor((int)x, 8);
            av &= x;
          }
          const uint32_t elig = av & ~ck_bits(0, il);
          if (elig) ks = ck_bond(__builtin_ctz(elig));
        }
        // the flipped amplitude over [f, ks), rows and columns meeting half
        // way; with all terms at once the first row step also leaves the
        // unflipped prefix extension in U
        const int c = meet(f, ks);
        if (!seq) {
          segment(f, c, c, ks, lj, j, true, 0, T);
          record(0, T);
        } else {
          for (int t = 0; t < T; ++t) {
            segment(f, c, c, ks, lj, j, false, t, 1);
            record(t, 1);
          }
        }
        int accept[CG];
#pragma unroll
        for (int cg = 0; cg < CG; ++cg) {
          accept[cg] = 0;
          if (live[cg] && stat[cg] == 0) {
            double lnew; int snew;
            amp(16 * cg + m, lnew, snew);
            if (isnan(lnew)) {
              stat[cg] = -5;
            } else if (snew != 0) {
              const double u = philox_uniform(a.seed, a.rstream, (uint64_t)(w0 + 16 * cg + m), sweep, (uint64_t)j);
              if (u < exp(2.0 * (lnew - lab[cg]))) {
                accept[cg] = 1;
                lab[cg] = lnew;
                sgn[cg] = snew;
                nacc[cg] += 1;
              }
            }
          }
        }
        // prefix through position f with the decided s_j
        if (!seq && side == 0) {  // each row lane copies the features it wrote in the first step
          for (int t = 0; t < T; ++t)
#pragma unroll
            for (int cg = 0; cg < CG; ++cg)
#pragma unroll
              for (int mt = 0; mt < MT; ++mt) {
                const int off = (16 * cg + m) * RS;
                A::copy4(buf(t, P) + off, buf(t, accept[cg] ? F : U) + off, 16 * (wv * MT + mt) + 4 * g);
              }
        }
        // checkpoints: the columns computed past lj hold the current
        // configuration for every walker; those at or before lj become the
        // saved ones of the walkers that accepted (copied by the 4 * nwave
        // lanes of each walker), and earlier ones at or before lj go stale
        // for them
        if (CKP && NCK > 0) {
          const int ic0 = ck_ceil(c), ic1 = ck_ceil(ks);  // computed: [ic0, ic1)
          const int icand = min(ic1, il);                  // candidates: [ic0, icand)
          const uint32_t past = ck_bits(max(ic0, il), ic1);
          const uint32_t cand = ck_bits(ic0, icand), stale = ck_bits(0, min(ic0, il));
          const int r = wave * 4 + g;  // index among a walker's lanes
#pragma unroll
          for (int cg = 0; cg < CG; ++cg) {
            vmask[cg] |= past;
            if (accept[cg]) {
              vmask[cg] = (vmask[cg] | cand) & ~stale;
              const int wn = 16 * cg + m;
              for (int i = ic0; i < icand; ++i)
                for (int t = 0; t < T; ++t) {
                  for (int q = r; q < CHI / 4; q += 4 * nwave) {
                    if constexpr (CKG)
                      __builtin_nontemporal_store(
                          __builtin_nontemporal_load(reinterpret_cast<const f4*>(gbuf(t, CD + i) + wn * RS) + q),
                          reinterpret_cast<f4*>(gbuf(t, CK + i) + wn * RS) + q);
                    else
                      reinterpret_cast<float4*>(buf(t, CK + i) + wn * RS)[q] =
                          reinterpret_cast<const float4*>(buf(t, CD + i) + wn * RS)[q];
                  }
                  if (r == 0) ckexp(CK + i, t, wn) = ckexp(CD + i, t, wn);
                }
            }
          }
        }
        if (wave == 0 && g == 0) {
#pragma unroll
          for (int cg = 0; cg < CG; ++cg) {
            const int wn = 16 * cg + m;
            if (!seq)
              for (int t = 0; t < T; ++t) Ep[t * NB + wn] = Ef[t * NB + wn];
            if (accept[cg]) {
              sp[wn * nw + (j >> 6)] ^= (1ull << (j & 63));
              for (int wd = 0; wd < LW; ++wd) pm[wn * LW + wd] ^= rword(j, wd);
            }
          }
        }
        __syncthreads();
        if (seq)  // one more step per term with the decided spin
          for (int t = 0; t < T; ++t) advance_prefix(f + 1, t, 1);
        pos = f + 1;
      }
    }
  }

  // write back
  if (wave == 0 && g == 0) {
#pragma unroll
    for (int cg = 0; cg < CG; ++cg) {
      if (!live[cg]) continue;
      const int wn = 16 * cg + m;
      const int w = w0 + wn;
      if (a.mode == 1)
        for (int wd = 0; wd < nw; ++wd) a.spins[(size_t)w * nw + wd] = sp[wn * nw + wd];
      const bool ok = stat[cg] == 0;
      if (a.logabs) a.logabs[w] = ok ? lab[cg] : NAN;
      if (a.sign) a.sign[w] = ok ? (int8_t)sgn[cg] : 0;
      if (a.accepts && a.mode == 1) a.accepts[w] += nacc[cg];
      if (a.status) a.status[w] = stat[cg];
    }
  }
}

template <class D, int CHI, int CG, bool CKP, bool CKG = false>
__global__ void __launch_bounds__((ChainGeo<CHI, D>::NT)) chain_kernel(ChainArgs a) {
  chain_body<D, CHI, CG, CKP, CKG>(a, blockIdx.x, a.sweep0);
}

// ============================================================================
// compensated reduction
// ============================================================================
__device__ __forceinline__ void neumaier_add(double& s, double& c, double x) {
  const double t = s + x;
  c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
  s = t;
}
__device__ __forceinline__ void neumaier_merge(double& s, double& c, double s2, double c2) {
  neumaier_add(s, c, s2);
  c += c2;
}

__device__ __forceinline__ void reduce_body(int n, const double* x, double* out) {
  __shared__ double sh[4][256];
  double s1 = 0, c1 = 0, s2 = 0, c2 = 0, cnt = 0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double v = x[i];
    if (!isfinite(v)) continue;
    neumaier_add(s1, c1, v);
    neumaier_add(s2, c2, v * v);
    cnt += 1.0;
  }
  sh[0][threadIdx.x] = s1; sh[1][threadIdx.x] = c1;
  sh[2][threadIdx.x] = s2; sh[3][threadIdx.x] = c2;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      double a1 = sh[0][threadIdx.x], b1 = sh[1][threadIdx.x];
      neumaier_merge(a1, b1, sh[0][threadIdx.x + off], sh[1][threadIdx.x + off]);
      double a2 = sh[2][threadIdx.x], b2 = sh[3][threadIdx.x];
      neumaier_merge(a2, b2, sh[2][threadIdx.x + off], sh[3][threadIdx.x + off]);
      sh[0][threadIdx.x] = a1; sh[1][threadIdx.x] = b1;
      sh[2][threadIdx.x] = a2; sh[3][threadIdx.x] = b2;
    }
    __syncthreads();
  }
  // counts are small integers: exact in double; reduce with a plain tree
  __shared__ double shc[256];
  shc[threadIdx.x] = cnt;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) shc[threadIdx.x] += shc[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sh[0][0] + sh[1][0];
    out[1] = sh[2][0] + sh[3][0];
    out[2] = shc[0];
  }
}

__global__ void __launch_bounds__(256) reduce_kernel(int n, const double* x, double* out) {
  reduce_body(n, x, out);
}

// Compensated FP64 sums of products of rows: block (a, b) sums x[a][w] *
// y[b][w] over w (y = null: x[a][w] alone) and counts the finite terms,
// out[2 (a B + b)] and out[2 (a B + b) + 1]; non-finite terms are skipped.
// The partial sums of the 256 threads meet in a fixed tree (deterministic).
__global__ void __launch_bounds__(256) pair_sums_kernel(int B, int W, const double* x, const double* y,
                                                        double* out) {
  __shared__ double sh[3][256];
  const int a = blockIdx.x / B, b = blockIdx.x % B;
  const double* xa = x + (size_t)a * W;
  const double* yb = y ? y + (size_t)b * W : nullptr;
  double s = 0, c = 0, cnt = 0;
  for (int i = threadIdx.x; i < W; i += 256) {
    const double v = yb ? xa[i] * yb[i] : xa[i];
    if (!isfinite(v)) continue;
    neumaier_add(s, c, v);
    cnt += 1.0;
  }
  sh[0][threadIdx.x] = s; sh[1][threadIdx.x] = c; sh[2][threadIdx.x] = cnt;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      double s1 = sh[0][threadIdx.x], c1 = sh[1][threadIdx.x];
      neumaier_merge(s1, c1, sh[0][threadIdx.x + off], sh[1][threadIdx.x + off]);
      sh[0][threadIdx.x] = s1; sh[1][threadIdx.x] = c1;
      sh[2][threadIdx.x] += sh[2][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * (size_t)blockIdx.x] = sh[0][0] + sh[1][0];
    out[2 * (size_t)blockIdx.x + 1] = sh[2][0];
  }
}

// ============================================================================
// persistent forms for batches of RTTs
// ============================================================================
// Work items (int4): x = descriptor index, y = block index within that
// descriptor's launch, z = term (pass kernel).  Blocks take items from a
// device counter until the list is exhausted; every wave reaches the exit.
__device__ __forceinline__ int next_item(int* counter, int* s_item) {
  if (threadIdx.x == 0) *s_item = atomicAdd(counter, 1);
  __syncthreads();
  const int it = *s_item;
  __syncthreads();
  return it;
}

template <class D, int CHI>
__global__ void __launch_bounds__(256, (pass_min_blocks<D, CHI>())) pass_persistent(const PassArgs* descs, const int4* items,
                                                       int n_items, int* counter) {
  __shared__ int s_item;
  for (;;) {
    const int it = next_item(counter, &s_item);
    if (it >= n_items) break;
    const int4 w = items[it];
    const PassArgs a = descs[w.x];
    pass_body<D, CHI>(a, w.y, w.z);
    __syncthreads();
  }
}

// CG column groups of 16 walkers per item (the batch autotuner's tile choice)
template <class D, int CHI, int CG>
__global__ void __launch_bounds__((ChainGeo<CHI, D>::NT)) chain_persistent(const ChainArgs* descs,
                                                                        const int4* items, int n_items,
                                                                        int* counter,
                                                                        const uint64_t* sweep0) {
  __shared__ int s_item;
  for (;;) {
    // uniform item index: the descriptor's fields are then scalar loads
    const int it = __builtin_amdgcn_readfirstlane(next_item(counter, &s_item));
    if (it >= n_items) break;
    const int4 w = items[it];
    chain_body<D, CHI, CG>(descs[w.x], w.y, *sweep0);
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) combine_persistent(const CombineArgs* descs, const int4* items,
                                                          int n_items, int* counter) {
  __shared__ int s_item;
  for (;;) {
    const int it = next_item(counter, &s_item);
    if (it >= n_items) break;
    const int4 w = items[it];
    const CombineArgs a = descs[w.x];
    combine_body(a, w.y);
    __syncthreads();
  }
}

// one block per RTT: out[3*b .. 3*b+2] = compensated sum, sum of squares, count
__global__ void __launch_bounds__(256) reduce_many(const int* n, const double* const* x, double* out) {
  reduce_body(n[blockIdx.x], x[blockIdx.x], out + 3 * blockIdx.x);
}

// Dual Monte Carlo estimators for one target state b, walkers sampled from
// P^a: ratio = psi^b / psi^a and the mixed local energy
// sum_t H_st psi^b(t) / psi^a(s) = ratio * E_loc^b(s), from both states'
// log|psi| and signs and b's local energy.  A walker whose sampled or target
// amplitude is zero or non-finite gets NaN and status -5; `first` starts the
// status, later targets fold into it.
__global__ void __launch_bounds__(256) mixed_kernel(int W, const double* la, const int8_t* sa,
                                                    const double* lb, const int8_t* sb, const double* eb,
                                                    const int32_t* stb, double* ratio, double* mixed,
                                                    int32_t* status, int first) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const bool ok = stb[w] == 0 && sa[w] != 0 && sb[w] != 0 && isfinite(la[w]) && isfinite(lb[w]) &&
                  isfinite(eb[w]);
  const double r = ok ? (double)(sa[w] * sb[w]) * exp(lb[w] - la[w]) : NAN;
  ratio[w] = r;
  mixed[w] = ok ? r * eb[w] : NAN;
  if (status) {
    const int32_t st = ok ? 0 : -5;
    status[w] = first ? st : min(status[w], st);
  }
}

// graph-safe clearing of work counters (a kernel, not a memset node)
__global__ void fill_int(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void advance_u64(uint64_t* p, uint64_t by) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p += by;
}

}  // namespace rttk
