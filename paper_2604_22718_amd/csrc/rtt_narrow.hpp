// Narrow-bond kernels: trains whose bonds are all at most 4 (the paper's
// chi = 2 states on the H+V+D+D' path are the case in point) contracted on
// the vector ALUs instead of 16 x 16 matrix-core tiles, which would pad a
// 2 x 2 core to 16 x 16 and waste 63/64 of the work.
//
// One thread carries one amplitude: a 1 x C row vector (C = 2 or 4) times
// the selected C x C slice of every position (Sec. 2.2.1 product).  Both
// slices of a position are read at addresses uniform across the wave
// (scalar loads); each lane forms both products and keeps the one its spin
// bit selects, so no lane branches.  The row is renormalised by a power of
// two every four positions (exact), its exponent kept as an integer, and
// terms of a linear combination (Sec. 3.2) are summed in FP64 at the end.
//
//   narrow_eval_kernel   one block per walker: thread j < N gives
//                        psi(s^j), thread N psi(s); flip ratios, log|psi|,
//                        sign and E_loc (Sec. 4 Ising Hamiltonian)
//   narrow_chain_kernel  one thread per walker: Metropolis sweeps (Sec. 3.3)
//                        in the proposal order, the unflipped prefix of the
//                        current spin's first position carried along
#pragma once
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>
#include <stdint.h>

#include "rtt_device.hpp"

namespace rttn {

constexpr int kNarrowMax = 4;   // widest bond taken by these kernels
constexpr int kMaxTermsN = 8;   // terms of a linear combination

struct NarrowArgs {
  const float* cores;      // [T][L][2][C][C] prescaled quantised cores, zero padded
  const int32_t* cesum;    // [T][L+1] prefix sums of the prescale exponents
  const uint64_t* rmask;   // [N][LW] train positions of each spin
  const int32_t* pi;       // [L]
  const int32_t* order;    // [N] proposal order
  const int32_t* first;    // [N] first position of each spin, -1 if unread
  const double* coeffs;    // [T]
  int T, L, N, nw, LW, W;
  const int2* bonds; int nbonds; double J, h;
  uint64_t* spins;
  double* logabs; int8_t* sign; double* logratio; int8_t* rsign; double* eloc;
  uint32_t* accepts; int32_t* status;
  uint64_t seed, rstream, sweep0;
  int n_sweeps, mode;
};

// x <- x 2^-e with e the exponent of max|x_i| (frexp convention), ex += e
template <int C>
__device__ __forceinline__ void renorm(float (&x)[C], int& ex) {
  float m = fabsf(x[0]);
#pragma unroll
  for (int c = 1; c < C; ++c) m = fmaxf(m, fabsf(x[c]));
  if (m == 0.f || !isfinite(m)) return;
  const int e = __builtin_amdgcn_frexp_expf(m);
#pragma unroll
  for (int c = 0; c < C; ++c) x[c] = ldexpf(x[c], -e);
  ex += e;
}

// One position: x <- x A[b], both slices formed, the bit's one kept.
template <int C>
__device__ __forceinline__ void step(const float* __restrict__ A, bool b, float (&x)[C]) {
  float y0[C], y1[C];
#pragma unroll
  for (int c = 0; c < C; ++c) { y0[c] = 0.f; y1[c] = 0.f; }
#pragma unroll
  for (int r = 0; r < C; ++r)
#pragma unroll
    for (int c = 0; c < C; ++c) {
      y0[c] = fmaf(x[r], A[r * C + c], y0[c]);
      y1[c] = fmaf(x[r], A[C * C + r * C + c], y1[c]);
    }
#pragma unroll
  for (int c = 0; c < C; ++c) x[c] = b ? y1[c] : y0[c];
}

// Row x (exponent ex) through positions [k0, k1) of one term's cores.  The
// slice bit of position k is bit k of the words bits(kw) (kw = k / 64).
// Renormalisation follows every position k with k % 4 == 3; the aligned
// groups of four run unrolled so that their slice loads issue together.
template <int C, class Bits>
__device__ __forceinline__ void advance(const float* __restrict__ tc, int k0, int k1, Bits bits, float (&x)[C],
                                        int& ex) {
  int k = k0;
  while (k < k1) {
    const int kw = k >> 6;
    const uint64_t word = bits(kw);
    const int kend = min(k1, (kw + 1) << 6);
    for (; k < kend && (k & 3); ++k) {
      step<C>(tc + (size_t)k * (2 * C * C), (word >> (k & 63)) & 1ull, x);
      if ((k & 3) == 3) renorm<C>(x, ex);
    }
    for (; k + 4 <= kend; k += 4) {
      const float* A = tc + (size_t)k * (2 * C * C);
      const uint32_t nib = (uint32_t)(word >> (k & 63));
#pragma unroll
      for (int i = 0; i < 4; ++i) step<C>(A + i * (2 * C * C), (nib >> i) & 1u, x);
      renorm<C>(x, ex);
    }
    for (; k < kend; ++k) step<C>(tc + (size_t)k * (2 * C * C), (word >> (k & 63)) & 1ull, x);
  }
}

template <int C>
__device__ __forceinline__ void unit_row(float (&x)[C], int& ex) {
#pragma unroll
  for (int c = 0; c < C; ++c) x[c] = c == 0 ? 1.f : 0.f;
  ex = 0;
}

// sum_t coeffs[t] m_t 2^e_t as (mant, ex), |mant| in [0.5, 1) or 0
__device__ __forceinline__ void combine_terms(int T, const double* coeffs, const float* m, const int* e,
                                              double& mant, int& ex) {
  int emax = INT_MIN;
  for (int t = 0; t < T; ++t)
    if (m[t] != 0.f && e[t] > emax) emax = e[t];
  if (emax == INT_MIN) { mant = 0.0; ex = 0; return; }
  double S = 0.0;
  for (int t = 0; t < T; ++t)
    if (m[t] != 0.f) S += ldexp(coeffs[t] * (double)m[t], e[t] - emax);
  int eS = 0;
  mant = frexp(S, &eS);
  ex = emax + eS;
}

// amplitude from position k0 on, every term starting from its row (xs, es)
template <int C, class Bits>
__device__ __forceinline__ void amplitude_from(const NarrowArgs& a, int k0, const float (*xs)[C], const int* es,
                                               Bits bits, double& mant, int& ex) {
  float m[kMaxTermsN];
  int e[kMaxTermsN];
  for (int t = 0; t < a.T; ++t) {
    float x[C];
    int xe = es[t];
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = xs[t][c];
    advance<C>(a.cores + (size_t)t * a.L * 2 * C * C, k0, a.L, bits, x, xe);
    m[t] = x[0];
    e[t] = xe + a.cesum[(size_t)t * (a.L + 1) + a.L];
  }
  combine_terms(a.T, a.coeffs, m, e, mant, ex);
}

__device__ __forceinline__ double block_sum(double x, double* red) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

// ---------------------------------------------------------------- evaluation
// Dynamic LDS: LW words of position bits.  blockDim.x = 64 * ceil((N+1)/64)
// capped at 1024, so that two rounds cover the N + 1 items for N <= 1024.
template <int C>
__global__ void __launch_bounds__(1024) narrow_eval_kernel(NarrowArgs a) {
  extern __shared__ uint64_t pm[];
  __shared__ double red[16];
  __shared__ double base_m;
  __shared__ int base_e;
  const int w = blockIdx.x;
  const uint64_t* sw = a.spins + (size_t)w * a.nw;
  for (int kw = threadIdx.x; kw < a.LW; kw += blockDim.x) {
    uint64_t word = 0;
    const int kend = min(a.L, (kw + 1) * 64);
    for (int k = kw * 64; k < kend; ++k) word |= (uint64_t)rttk::spin_bit(sw, a.pi[k]) << (k & 63);
    pm[kw] = word;
  }
  __syncthreads();
  float x0[kMaxTermsN][C];
  int e0[kMaxTermsN];
  for (int t = 0; t < a.T; ++t) unit_row<C>(x0[t], e0[t]);
  // items 0..N-1 are the flipped configurations, item N the configuration
  // itself; a thread takes items threadIdx.x and threadIdx.x + blockDim.x
  double mi[2] = {0.0, 0.0};
  int ei[2] = {0, 0};
  for (int it = 0; it < 2; ++it) {
    const int item = threadIdx.x + it * blockDim.x;
    if (item > a.N) break;
    if (item < a.N && a.first[item] < 0) continue;
    // one code path for every lane: the configuration itself flips nothing
    const uint64_t* xm = item < a.N ? a.rmask + (size_t)item * a.LW : nullptr;
    amplitude_from<C>(a, 0, x0, e0, [&](int kw) { return pm[kw] ^ (xm ? xm[kw] : 0ull); }, mi[it], ei[it]);
    if (item == a.N) {
      base_m = mi[it];
      base_e = ei[it];
    }
  }
  __syncthreads();
  const double m0 = base_m;
  const int ebase = base_e;
  const bool ok = m0 != 0.0 && isfinite(m0);
  const double LN2 = 0.69314718055994530942;
  double rsum = 0.0;
  for (int it = 0; it < 2; ++it) {
    const int j = threadIdx.x + it * blockDim.x;
    if (j >= a.N) break;
    double lr = NAN, r = NAN;
    int8_t sg = 0;
    if (ok) {
      if (a.first[j] < 0) {  // spin read by no position: r_j = 1 exactly
        lr = 0.0; sg = 1; r = 1.0;
      } else if (mi[it] == 0.0) {
        lr = -INFINITY; sg = 1; r = 0.0;
      } else {
        lr = log(fabs(mi[it])) - log(fabs(m0)) + (double)(ei[it] - ebase) * LN2;
        sg = ((mi[it] > 0) == (m0 > 0)) ? 1 : -1;
        r = sg * exp(lr);
      }
      rsum += r;
    }
    if (a.logratio) a.logratio[(size_t)w * a.N + j] = lr;
    if (a.rsign) a.rsign[(size_t)w * a.N + j] = sg;
  }
  if (a.eloc) {
    double diag = 0.0;
    for (int b = threadIdx.x; b < a.nbonds; b += blockDim.x) {
      const int2 bd = a.bonds[b];
      diag += (rttk::spin_bit(sw, bd.x) ^ rttk::spin_bit(sw, bd.y)) ? -1.0 : 1.0;
    }
    diag = block_sum(diag, red);
    rsum = block_sum(rsum, red);
    if (threadIdx.x == 0) a.eloc[w] = ok ? a.J * diag - a.h * rsum : NAN;
  }
  if (threadIdx.x == 0) {
    if (a.logabs) a.logabs[w] = ok ? log(fabs(m0)) + ebase * LN2 : NAN;
    if (a.sign) a.sign[w] = ok ? (m0 > 0 ? 1 : -1) : 0;
    if (a.status) a.status[w] = ok ? 0 : -5;
  }
}

// ---------------------------------------------------------------- sampling
// 64 walkers per block, one per lane.  Dynamic LDS: position bits [LW][64]
// and spin words [nw][64] of the block's walkers.
template <int C>
__global__ void __launch_bounds__(64) narrow_chain_kernel(NarrowArgs a) {
  extern __shared__ uint64_t sh[];
  uint64_t* pm = sh;
  uint64_t* sp = sh + (size_t)a.LW * 64;
  const int lane = threadIdx.x;
  const int w = blockIdx.x * 64 + lane;
  const bool live = w < a.W;
  for (int wd = 0; wd < a.nw; ++wd) sp[wd * 64 + lane] = live ? a.spins[(size_t)w * a.nw + wd] : 0ull;
  for (int kw = 0; kw < a.LW; ++kw) {
    uint64_t word = 0;
    const int kend = min(a.L, (kw + 1) * 64);
    for (int k = kw * 64; k < kend; ++k) {
      const int q = a.pi[k];
      word |= ((sp[(q >> 6) * 64 + lane] >> (q & 63)) & 1ull) << (k & 63);
    }
    pm[kw * 64 + lane] = word;
  }
  auto cur = [&](int kw) { return pm[kw * 64 + lane]; };
  float xp[kMaxTermsN][C];   // unflipped prefix rows through position pos
  int ep[kMaxTermsN];
  for (int t = 0; t < a.T; ++t) unit_row<C>(xp[t], ep[t]);
  double m0; int e0;
  amplitude_from<C>(a, 0, xp, ep, cur, m0, e0);
  const double LN2 = 0.69314718055994530942;
  int stat = (m0 != 0.0 && isfinite(m0)) ? 0 : -5;
  double lab = stat == 0 ? log(fabs(m0)) + e0 * LN2 : NAN;
  int sgn = stat == 0 ? (m0 > 0 ? 1 : -1) : 0;
  uint32_t nacc = 0;
  if (a.mode == 1) {
    for (int ts = 0; ts < a.n_sweeps; ++ts) {
      const uint64_t sweep = a.sweep0 + (uint64_t)ts;
      for (int t = 0; t < a.T; ++t) unit_row<C>(xp[t], ep[t]);
      int pos = 0;
      for (int qi = 0; qi < a.N; ++qi) {
        const int j = a.order[qi];
        const int f = a.first[j];
        if (f < 0) {  // spin read by no position: ratio 1, always accepted
          if (live && stat == 0) {
            nacc += 1;
            sp[(j >> 6) * 64 + lane] ^= 1ull << (j & 63);
          }
          continue;
        }
        for (int t = 0; t < a.T; ++t)
          advance<C>(a.cores + (size_t)t * a.L * 2 * C * C, pos, f, cur, xp[t], ep[t]);
        pos = f;
        const uint64_t* xm = a.rmask + (size_t)j * a.LW;
        double mj; int ej;
        amplitude_from<C>(a, f, xp, ep, [&](int kw) { return pm[kw * 64 + lane] ^ xm[kw]; }, mj, ej);
        if (live && stat == 0) {
          if (!isfinite(mj)) {
            stat = -5;
          } else if (mj != 0.0) {
            const double lnew = log(fabs(mj)) + ej * LN2;
            const double u = rttk::philox_uniform(a.seed, a.rstream, (uint64_t)w, sweep, (uint64_t)j);
            if (u < exp(2.0 * (lnew - lab))) {
              lab = lnew;
              sgn = mj > 0 ? 1 : -1;
              nacc += 1;
              sp[(j >> 6) * 64 + lane] ^= 1ull << (j & 63);
              for (int kw = 0; kw < a.LW; ++kw) pm[kw * 64 + lane] ^= xm[kw];
            }
          }
        }
      }
    }
  }
  if (!live) return;
  if (a.mode == 1)
    for (int wd = 0; wd < a.nw; ++wd) a.spins[(size_t)w * a.nw + wd] = sp[wd * 64 + lane];
  const bool ok = stat == 0;
  if (a.logabs) a.logabs[w] = ok ? lab : NAN;
  if (a.sign) a.sign[w] = ok ? (int8_t)sgn : 0;
  if (a.accepts && a.mode == 1) a.accepts[w] += nacc;
  if (a.status) a.status[w] = stat;
}

}  // namespace rttn

namespace rttn {

// ---------------------------------------------------------------- segmented sampling
// G lanes per walker (64 / G walkers per wave), lane g owning the positions
// [g S, g S + S) (S = ceil(L / G) <= 64, their slice bits in one register
// word) and the C x C product of its segment for the current configuration.
// A proposal recomputes only the segments that hold a replica of the spin;
// the G products meet in a log2(G)-level tree across lanes, and the walker's
// lane g = 0 decides.  One term only.  Dynamic LDS: the C x C slices of all
// positions (shared by the block's walkers), then the spin words.
template <int C>
struct SegMat {
  float m[C * C];
  int e;
};

template <int C>
__device__ __forceinline__ void seg_renorm(SegMat<C>& M) {
  float mx = 0.f;
#pragma unroll
  for (int i = 0; i < C * C; ++i) mx = fmaxf(mx, fabsf(M.m[i]));
  if (mx == 0.f || !isfinite(mx)) return;
  const int e = __builtin_amdgcn_frexp_expf(mx);
#pragma unroll
  for (int i = 0; i < C * C; ++i) M.m[i] = ldexpf(M.m[i], -e);
  M.e += e;
}

// product of positions [k0, k0 + len) with slice bits `bits` (bit i for k0 + i)
template <int C>
__device__ __forceinline__ SegMat<C> seg_product(const float* __restrict__ lc, int k0, int len, uint64_t bits) {
  SegMat<C> M;
#pragma unroll
  for (int i = 0; i < C * C; ++i) M.m[i] = (i / C == i % C) ? 1.f : 0.f;
  M.e = 0;
  for (int i = 0; i < len; ++i) {
    const float* A = lc + (size_t)(k0 + i) * (2 * C * C);
    float a0[C * C], a1[C * C];
#pragma unroll
    for (int q = 0; q < C * C; ++q) { a0[q] = A[q]; a1[q] = A[C * C + q]; }
    const bool b = (bits >> i) & 1ull;
#pragma unroll
    for (int r = 0; r < C; ++r) {
      float y0[C], y1[C];
#pragma unroll
      for (int c = 0; c < C; ++c) { y0[c] = 0.f; y1[c] = 0.f; }
#pragma unroll
      for (int q = 0; q < C; ++q)
#pragma unroll
        for (int c = 0; c < C; ++c) {
          y0[c] = fmaf(M.m[r * C + q], a0[q * C + c], y0[c]);
          y1[c] = fmaf(M.m[r * C + q], a1[q * C + c], y1[c]);
        }
#pragma unroll
      for (int c = 0; c < C; ++c) M.m[r * C + c] = b ? y1[c] : y0[c];
    }
    if ((i & 3) == 3) seg_renorm<C>(M);
  }
  seg_renorm<C>(M);
  return M;
}

// bits [k0, k0 + len) of a position mask stored as 64-bit words
__device__ __forceinline__ uint64_t mask_bits(const uint64_t* words, int LW, int k0, int len) {
  if (len <= 0) return 0ull;
  const int w0 = k0 >> 6, sh = k0 & 63;
  uint64_t v = words[w0] >> sh;
  if (sh && w0 + 1 < LW) v |= words[w0 + 1] << (64 - sh);
  return len >= 64 ? v : (v & ((1ull << len) - 1ull));
}

// product of the walker's G segment matrices (lanes g = 0..G-1, in order);
// the result is valid in lane g = 0
template <int C, int G>
__device__ __forceinline__ SegMat<C> seg_tree(SegMat<C> M, int g) {
#pragma unroll
  for (int d = 1; d < G; d <<= 1) {
    SegMat<C> O;
#pragma unroll
    for (int i = 0; i < C * C; ++i) O.m[i] = __shfl_down(M.m[i], d, 64);
    O.e = __shfl_down(M.e, d, 64);
    if ((g & (2 * d - 1)) == 0) {
      SegMat<C> P;
#pragma unroll
      for (int r = 0; r < C; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) {
          float acc = 0.f;
#pragma unroll
          for (int q = 0; q < C; ++q) acc = fmaf(M.m[r * C + q], O.m[q * C + c], acc);
          P.m[r * C + c] = acc;
        }
      P.e = M.e + O.e;
      seg_renorm<C>(P);
      M = P;
    }
  }
  return M;
}

template <int C, int G>
__global__ void __launch_bounds__(64) narrow_chain_seg_kernel(NarrowArgs a) {
  extern __shared__ uint64_t shs[];
  float* lc = reinterpret_cast<float*>(shs);                          // [L][2][C][C]
  const size_t cw = ((size_t)a.L * 2 * C * C * 4 + 7) / 8;
  uint64_t* sp = shs + cw;                                            // [64 / G][nw]
  constexpr int WPB = 64 / G;
  const int lane = threadIdx.x;
  const int ws = lane / G, g = lane % G;
  const int w = blockIdx.x * WPB + ws;
  const bool live = w < a.W;
  for (int i = lane; i < a.L * 2 * C * C; i += 64) lc[i] = a.cores[i];
  for (int i = lane; i < WPB * a.nw; i += 64) {
    const int wv = blockIdx.x * WPB + i / a.nw;
    sp[i] = wv < a.W ? a.spins[(size_t)wv * a.nw + i % a.nw] : 0ull;
  }
  __syncthreads();
  const int S = (a.L + G - 1) / G;
  const int k0 = g * S;
  const int len = max(0, min(a.L, k0 + S) - k0);
  uint64_t* spw = sp + ws * a.nw;
  uint64_t pw = 0;
  for (int i = 0; i < len; ++i) {
    const int q = a.pi[k0 + i];
    pw |= ((spw[q >> 6] >> (q & 63)) & 1ull) << i;
  }
  SegMat<C> M = seg_product<C>(lc, k0, len, pw);
  const int esum = a.cesum[a.L];
  const double LN2 = 0.69314718055994530942;
  auto amp = [&](const SegMat<C>& T0, double& lab_out, int& sg_out) {  // lane g = 0
    const double m = (double)T0.m[0] * a.coeffs[0];
    if (m == 0.0 || !isfinite(m)) { lab_out = m == 0.0 ? -INFINITY : NAN; sg_out = 0; return; }
    lab_out = log(fabs(m)) + (double)(T0.e + esum) * LN2;
    sg_out = m > 0 ? 1 : -1;
  };
  double lab = NAN;
  int sgn = 0, stat = 0;
  {
    const SegMat<C> T0 = seg_tree<C, G>(M, g);
    amp(T0, lab, sgn);
    stat = (sgn != 0 && isfinite(lab)) ? 0 : -5;
  }
  uint32_t nacc = 0;
  if (a.mode == 1) {
    for (int ts = 0; ts < a.n_sweeps; ++ts) {
      const uint64_t sweep = a.sweep0 + (uint64_t)ts;
      for (int qi = 0; qi < a.N; ++qi) {
        const int j = a.order[qi];
        if (a.first[j] < 0) {  // spin read by no position: ratio 1, always accepted
          if (g == 0 && live && stat == 0) {
            nacc += 1;
            spw[j >> 6] ^= 1ull << (j & 63);
          }
          continue;
        }
        const uint64_t fm = mask_bits(a.rmask + (size_t)j * a.LW, a.LW, k0, len);
        SegMat<C> Mp = M;
        if (fm) Mp = seg_product<C>(lc, k0, len, pw ^ fm);
        const SegMat<C> T1 = seg_tree<C, G>(Mp, g);
        int accept = 0;
        if (g == 0 && live && stat == 0) {
          double lnew; int snew;
          amp(T1, lnew, snew);
          if (isnan(lnew)) {
            stat = -5;
          } else if (snew != 0) {
            const double u = rttk::philox_uniform(a.seed, a.rstream, (uint64_t)w, sweep, (uint64_t)j);
            if (u < exp(2.0 * (lnew - lab))) {
              accept = 1;
              lab = lnew;
              sgn = snew;
              nacc += 1;
              spw[j >> 6] ^= 1ull << (j & 63);
            }
          }
        }
        accept = __shfl(accept, ws * G, 64);
        if (accept && fm) {
          M = Mp;
          pw ^= fm;
        }
      }
    }
  }
  __syncthreads();
  if (!live || g != 0) return;
  if (a.mode == 1)
    for (int wd = 0; wd < a.nw; ++wd) a.spins[(size_t)w * a.nw + wd] = spw[wd];
  const bool ok = stat == 0;
  if (a.logabs) a.logabs[w] = ok ? lab : NAN;
  if (a.sign) a.sign[w] = ok ? (int8_t)sgn : 0;
  if (a.accepts && a.mode == 1) a.accepts[w] += nacc;
  if (a.status) a.status[w] = stat;
}

}  // namespace rttn
