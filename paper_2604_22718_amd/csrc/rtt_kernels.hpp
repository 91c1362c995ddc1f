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
//                  amplitudes, and Metropolis sweeps with Philox uniforms.
//  reduce_kernel   compensated FP64 sums of local energies.
#pragma once
#include <float.h>
#include <math.h>

#include "rtt_device.hpp"

namespace rttk {

constexpr int kMaxTerms = 8;

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
  const int4* sched;
  int n_steps;
  int nslot;                // rows per walker, multiple of 16
  int L, nw, W;
  const uint64_t* spins;    // [W][nw]
  float* out_vec;           // [T][W][nslot][CHI]
  int32_t* out_exp;         // [T][W][nslot]
};

template <class D, int CHI>
__global__ void __launch_bounds__(256) pass_kernel(PassArgs a) {
  using E = typename D::elem;
  using G = Geo<CHI>;
  constexpr int WPW = G::WPW, MT = G::MT, KPL = G::KPL, RS = G::RS;
  constexpr int WPB = 4 / WPW;
  extern __shared__ __align__(16) float lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ws = wave / WPW, wv = wave % WPW;
  const int g = lane >> 4, m = lane & 15;
  const int term = blockIdx.y;
  const int w_raw = blockIdx.x * WPB + ws;
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
  if (tid_w == 0) cur[0] = 1.f;  // boundary vector e_0 in the base slot
  __syncthreads();

  const E* cores = static_cast<const E*>(a.cores) + (size_t)term * a.L * 2 * CHI * CHI;
  const int* cexp_p = a.core_exp ? a.core_exp + (size_t)term * a.L : nullptr;

  for (int s = 0; s < a.n_steps; ++s) {
    const int4 st = a.sched[s];
    const int k = st.x, q = st.y, nact = st.z, odd = st.w;
    const int bit = spin_bit(spw, q);
    const E* Am = cores + ((size_t)k * 2 + bit) * (CHI * CHI) + (size_t)lane * KPL;
    const E* Ao = cores + ((size_t)k * 2 + (bit ^ 1)) * (CHI * CHI) + (size_t)lane * KPL;
    E fm[MT][KPL], fo[MT][KPL];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int t = wv * MT + mt;
      load_frag<KPL>(fm[mt], Am + (size_t)t * 64 * KPL);
      load_frag<KPL>(fo[mt], Ao + (size_t)t * 64 * KPL);
    }
    const int cexp = cexp_p ? cexp_p[k] : 0;
    const int ntile = (nact + 15) >> 4;
    for (int r = 0; r < ntile; ++r) {
      const int row = 16 * r + m;
      float v[KPL];
      lds_read<KPL>(v, cur + row * RS + g * KPL);
      const int e = renorm_row<KPL>(v);
      if (wv == 0 && g == 0) exn[row] = exc[row] + e + cexp;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int t = wv * MT + mt;
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = D::template tile<KPL>(fm[mt], v, acc);
        *reinterpret_cast<float4*>(nxt + row * RS + 16 * t + 4 * g) =
            make_float4(acc[0], acc[1], acc[2], acc[3]);
      }
    }
    {  // odd row on the vector ALUs: out[16t+m] = sum_k A[1-s][k][16t+m] in[k]
      const int oin = odd & 0xffff, oout = odd >> 16;
      float v[KPL];
      lds_read<KPL>(v, cur + oin * RS + g * KPL);
      const int e = renorm_row<KPL>(v);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int t = wv * MT + mt;
        float p = 0.f;
#pragma unroll
        for (int c = 0; c < KPL; ++c) p = fmaf(D::to_f32(fo[mt][c]), v[c], p);
        p += __shfl_xor(p, 16);
        p += __shfl_xor(p, 32);
        if (g == 0) nxt[oout * RS + 16 * t + m] = p;
      }
      if (wv == 0 && lane == 0) exn[oout] = exc[oin] + e + cexp;
    }
    __syncthreads();
    float* tp = cur; cur = nxt; nxt = tp;
    int* te = exc; exc = exn; exn = te;
  }

  if (w_raw < a.W) {
    float* ov = a.out_vec + (((size_t)term * a.W + w) * nslot) * CHI;
    for (int i = tid_w; i < nslot * CHI; i += NT_W) ov[i] = cur[(i / CHI) * RS + (i % CHI)];
    int32_t* oe = a.out_exp + ((size_t)term * a.W + w) * nslot;
    for (int i = tid_w; i < nslot; i += NT_W) oe[i] = exc[i];
  }
}

// ============================================================================
// combine kernel (one wave per walker)
// ============================================================================
struct CombineArgs {
  const float* u; const int32_t* ue;  // forward  [T][W][nsf][chi], [T][W][nsf]
  const float* v; const int32_t* ve;  // backward [T][W][nsb][chi], [T][W][nsb]
  int nsf, nsb, chi, T, W, N, nw;
  const int32_t* fslot;               // [N] forward slot of spin j (0 = base)
  const int32_t* bslot;               // [N] backward slot of spin j (0 = base)
  const double* coeffs;               // [T]
  const uint64_t* spins;
  const int2* bonds; int nbonds; double J, h;
  double* logabs; int8_t* sign; double* logratio; int8_t* rsign; double* eloc; int32_t* status;
};

// value = mant * 2^ex with |mant| in [0.5, 1) (mant = 0 for zero)
__device__ inline void combined_value(const CombineArgs& a, int w, int fs, int bs, double& mant,
                                      int& ex) {
  double ms[kMaxTerms];
  int es[kMaxTerms];
  int emax = INT_MIN;
  for (int t = 0; t < a.T; ++t) {
    const float* pu = a.u + (((size_t)t * a.W + w) * a.nsf + fs) * a.chi;
    const float* pv = a.v + (((size_t)t * a.W + w) * a.nsb + bs) * a.chi;
    double d = 0.0;
    for (int f = 0; f < a.chi; f += 4) {
      const float4 x = *reinterpret_cast<const float4*>(pu + f);
      const float4 y = *reinterpret_cast<const float4*>(pv + f);
      d = fma((double)x.x, (double)y.x, d);
      d = fma((double)x.y, (double)y.y, d);
      d = fma((double)x.z, (double)y.z, d);
      d = fma((double)x.w, (double)y.w, d);
    }
    int ed = 0;
    const double md = frexp(d, &ed);
    ms[t] = a.coeffs[t] * md;
    es[t] = a.ue[((size_t)t * a.W + w) * a.nsf + fs] + a.ve[((size_t)t * a.W + w) * a.nsb + bs] + ed;
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

__global__ void __launch_bounds__(256) combine_kernel(CombineArgs a) {
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= a.W) return;
  const double LN2 = 0.69314718055994530942;
  double m0; int e0;
  combined_value(a, w, 0, 0, m0, e0);
  const bool ok = (m0 != 0.0) && isfinite(m0);
  const double lab0 = ok ? log(fabs(m0)) + e0 * LN2 : NAN;
  if (lane == 0) {
    if (a.logabs) a.logabs[w] = lab0;
    if (a.sign) a.sign[w] = ok ? (m0 > 0 ? 1 : -1) : 0;
    if (a.status) a.status[w] = ok ? 0 : -5;
  }
  double rsum = 0.0;
  for (int j = lane; j < a.N; j += 64) {
    const int fs = a.fslot[j], bs = a.bslot[j];
    double lr = NAN, r = NAN;
    int8_t sg = 0;
    if (ok) {
      if (fs == 0 && bs == 0) {  // spin read by no position: r_j = 1 exactly
        lr = 0.0; sg = 1; r = 1.0;
      } else {
        double mj; int ej;
        combined_value(a, w, fs, bs, mj, ej);
        if (mj == 0.0) { lr = -INFINITY; sg = 1; r = 0.0; }
        else {
          lr = log(fabs(mj)) - log(fabs(m0)) + (double)(ej - e0) * LN2;
          sg = ((mj > 0) == (m0 > 0)) ? 1 : -1;
          r = sg * exp(lr);
        }
      }
    }
    if (a.logratio) a.logratio[(size_t)w * a.N + j] = lr;
    if (a.rsign) a.rsign[(size_t)w * a.N + j] = sg;
    rsum += ok ? r : 0.0;
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

// ============================================================================
// chain kernel: 16 walkers per block, amplitudes and Metropolis sweeps
// ============================================================================
struct ChainArgs {
  const void* cores;        // [T][L][2][CHI*CHI] forward fragment layout
  const int32_t* core_exp;  // [T][L] or null
  const int32_t* pi;        // [L]
  const int32_t* order;     // [N] proposal order
  const int32_t* first;     // [N] first position of spin j, -1 if none
  const double* coeffs;     // [T]
  int T, L, N, nw, W;
  uint64_t* spins;
  double* logabs; int8_t* sign; uint32_t* accepts; int32_t* status;
  uint64_t seed, rstream, sweep0;
  int n_sweeps;
  int mode;                 // 0: amplitudes only, 1: sweeps
};

template <int CHI>
struct ChainLds {
  // per term: 5 row buffers (P prefix, U unflipped first step, F flipped
  // first step, X/Y ping-pong) of 16 rows, and 5 x 16 exponents
  static constexpr int kBufs = 5;
  static constexpr int rows_floats() { return kBufs * 16 * Geo<CHI>::RS; }
};

// One step for all 16 walkers (columns) of one term: both slices are applied
// and each column keeps the slice of its own walker.  out2 (optional)
// receives the other slice's product.
template <class D, int CHI>
__device__ __forceinline__ void chain_step(const typename D::elem* A0, const typename D::elem* A1,
                                           int cexp, const float* in, const int* ein, float* out,
                                           int* eout, float* out2, int* eout2, int bitn, int wv,
                                           int lane) {
  using G = Geo<CHI>;
  constexpr int MT = G::MT, KPL = G::KPL, RS = G::RS;
  const int g = lane >> 4, m = lane & 15;
  float v[KPL];
  lds_read<KPL>(v, in + m * RS + g * KPL);
  const int e = renorm_row<KPL>(v);
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int t = wv * MT + mt;
    typename D::elem f0[KPL], f1[KPL];
    load_frag<KPL>(f0, A0 + ((size_t)t * 64 + lane) * KPL);
    load_frag<KPL>(f1, A1 + ((size_t)t * 64 + lane) * KPL);
    f4 z = {0.f, 0.f, 0.f, 0.f};
    const f4 a0 = D::template tile<KPL>(f0, v, z);
    const f4 a1 = D::template tile<KPL>(f1, v, z);
    const f4 sel = bitn ? a1 : a0;
    *reinterpret_cast<float4*>(out + m * RS + 16 * t + 4 * g) = make_float4(sel[0], sel[1], sel[2], sel[3]);
    if (out2) {
      const f4 oth = bitn ? a0 : a1;
      *reinterpret_cast<float4*>(out2 + m * RS + 16 * t + 4 * g) =
          make_float4(oth[0], oth[1], oth[2], oth[3]);
    }
  }
  if (wv == 0 && g == 0) {
    eout[m] = ein[m] + e + cexp;
    if (eout2) eout2[m] = ein[m] + e + cexp;
  }
}

template <class D, int CHI>
__global__ void __launch_bounds__(64 * Geo<CHI>::WPW) chain_kernel(ChainArgs a) {
  using E = typename D::elem;
  using G = Geo<CHI>;
  constexpr int RS = G::RS;
  constexpr int BUF = 16 * RS;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m = lane & 15;
  const int nthr = blockDim.x;
  extern __shared__ __align__(16) float lds[];
  const int T = a.T;
  float* rows = lds;                                                  // [T][5][16][RS]
  int* exps = reinterpret_cast<int*>(lds + T * 5 * BUF);              // [T][5][16]
  uint64_t* sp = reinterpret_cast<uint64_t*>(exps + T * 5 * 16 + ((T * 5 * 16) & 1));  // [16][nw]
  double* lab = reinterpret_cast<double*>(sp + 16 * a.nw);            // [16] log|psi|
  int* sgn = reinterpret_cast<int*>(lab + 16);                        // [16]
  int* stat = sgn + 16;                                               // [16]
  int* flag = stat + 16;                                              // [16]
  uint32_t* acc = reinterpret_cast<uint32_t*>(flag + 16);             // [16]

  enum { P = 0, U = 1, F = 2, X = 3, Y = 4 };
  auto buf = [&](int t, int b) { return rows + (t * 5 + b) * BUF; };
  auto ebuf = [&](int t, int b) { return exps + (t * 5 + b) * 16; };

  const int w0 = blockIdx.x * 16;
  for (int i = threadIdx.x; i < T * 5 * BUF; i += nthr) rows[i] = 0.f;
  for (int i = threadIdx.x; i < T * 5 * 16; i += nthr) exps[i] = 0;
  for (int i = threadIdx.x; i < 16 * a.nw; i += nthr) {
    const int n = i / a.nw, wd = i % a.nw;
    sp[i] = (w0 + n < a.W) ? a.spins[(size_t)(w0 + n) * a.nw + wd] : 0ull;
  }
  if (threadIdx.x < 16) {
    acc[threadIdx.x] = 0;
    stat[threadIdx.x] = 0;
  }
  __syncthreads();

  const E* cores = static_cast<const E*>(a.cores);
  auto slice = [&](int t, int k, int b) {
    return cores + (((size_t)t * a.L + k) * 2 + b) * (CHI * CHI);
  };
  auto cexp_of = [&](int t, int k) { return a.core_exp ? a.core_exp[(size_t)t * a.L + k] : 0; };

  // reset the prefix of every term to the left boundary vector e_0
  auto reset_prefix = [&]() {
    for (int i = threadIdx.x; i < T * 16 * RS; i += nthr) {
      const int t = i / (16 * RS), r = i % (16 * RS);
      buf(t, P)[r] = (r % RS == 0) ? 1.f : 0.f;
    }
    for (int i = threadIdx.x; i < T * 16; i += nthr) ebuf(i / 16, P)[i % 16] = 0;
  };

  // advance rows in buffer `from` through positions [k0, k1) with spin jflip
  // flipped; returns the buffer index holding the result (X or Y)
  auto run = [&](int from, int k0, int k1, int jflip) {
    int cur = from;
    for (int k = k0; k < k1; ++k) {
      const int q = a.pi[k];
      const int bitn = spin_bit(sp + m * a.nw, q) ^ (q == jflip ? 1 : 0);
      const int nxt = (cur == X) ? Y : X;
      for (int t = 0; t < T; ++t)
        chain_step<D, CHI>(slice(t, k, 0), slice(t, k, 1), cexp_of(t, k), buf(t, cur),
                           ebuf(t, cur), buf(t, nxt), ebuf(t, nxt), nullptr, nullptr, bitn, wv,
                           lane);
      __syncthreads();
      cur = nxt;
    }
    return cur;
  };

  // combined amplitude of walker n from feature 0 of buffer b of every term
  auto amp = [&](int b, int n, double& labs, int& sg) {
    double ms[kMaxTerms];
    int es[kMaxTerms];
    int emax = INT_MIN;
    for (int t = 0; t < T; ++t) {
      int ed = 0;
      const double md = frexp((double)buf(t, b)[n * RS], &ed);
      ms[t] = a.coeffs[t] * md;
      es[t] = ebuf(t, b)[n] + ed;
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

  // amplitude of the current configuration
  reset_prefix();
  __syncthreads();
  {
    const int fin = run(P, 0, a.L, -1);
    if (threadIdx.x < 16) {
      double l; int s;
      amp(fin, threadIdx.x, l, s);
      lab[threadIdx.x] = l;
      sgn[threadIdx.x] = s;
      stat[threadIdx.x] = (s != 0 && isfinite(l)) ? 0 : -5;
    }
    __syncthreads();
  }

  if (a.mode == 1) {
    for (int ts = 0; ts < a.n_sweeps; ++ts) {
      const uint64_t sweep = a.sweep0 + (uint64_t)ts;
      reset_prefix();
      __syncthreads();
      int pos = 0;
      for (int qi = 0; qi < a.N; ++qi) {
        const int j = a.order[qi];
        const int f = a.first[j];
        if (f < 0) {  // spin read by no position: ratio 1, always accepted
          if (threadIdx.x < 16 && w0 + threadIdx.x < a.W && stat[threadIdx.x] == 0) {
            sp[threadIdx.x * a.nw + (j >> 6)] ^= (1ull << (j & 63));
            acc[threadIdx.x] += 1;
          }
          __syncthreads();
          continue;
        }
        if (pos < f) {  // bring the prefix up to position f
          const int fin = run(P, pos, f, -1);
          for (int i = threadIdx.x; i < T * 16 * RS; i += nthr) {
            const int t = i / (16 * RS), r = i % (16 * RS);
            buf(t, P)[r] = buf(t, fin)[r];
          }
          for (int i = threadIdx.x; i < T * 16; i += nthr) ebuf(i / 16, P)[i % 16] = ebuf(i / 16, fin)[i % 16];
          __syncthreads();
        }
        {  // first step at f: F gets the flipped slice, U the current one
          const int bitn = spin_bit(sp + m * a.nw, j) ^ 1;
          for (int t = 0; t < T; ++t)
            chain_step<D, CHI>(slice(t, f, 0), slice(t, f, 1), cexp_of(t, f), buf(t, P), ebuf(t, P),
                               buf(t, F), ebuf(t, F), buf(t, U), ebuf(t, U), bitn, wv, lane);
          __syncthreads();
        }
        int fin = F;
        if (f + 1 < a.L) {
          // run() ping-pongs X/Y; start from F by copying nothing: step F -> X first
          int cur = F;
          for (int k = f + 1; k < a.L; ++k) {
            const int q = a.pi[k];
            const int bitn = spin_bit(sp + m * a.nw, q) ^ (q == j ? 1 : 0);
            const int nxt = (cur == X) ? Y : X;
            for (int t = 0; t < T; ++t)
              chain_step<D, CHI>(slice(t, k, 0), slice(t, k, 1), cexp_of(t, k), buf(t, cur),
                                 ebuf(t, cur), buf(t, nxt), ebuf(t, nxt), nullptr, nullptr, bitn,
                                 wv, lane);
            __syncthreads();
            cur = nxt;
          }
          fin = cur;
        }
        if (threadIdx.x < 16) {
          const int n = threadIdx.x;
          int accept = 0;
          if (w0 + n < a.W && stat[n] == 0) {
            double lnew; int snew;
            amp(fin, n, lnew, snew);
            if (isnan(lnew)) {
              stat[n] = -5;
            } else if (snew != 0) {
              const double u = philox_uniform(a.seed, a.rstream, (uint64_t)(w0 + n), sweep, (uint64_t)j);
              const double r2 = exp(2.0 * (lnew - lab[n]));
              if (u < r2) {
                accept = 1;
                sp[n * a.nw + (j >> 6)] ^= (1ull << (j & 63));
                lab[n] = lnew;
                sgn[n] = snew;
                acc[n] += 1;
              }
            }
          }
          flag[n] = accept;
        }
        __syncthreads();
        // prefix through position f with the decided value of s_j
        for (int i = threadIdx.x; i < T * 16 * RS; i += nthr) {
          const int t = i / (16 * RS), r = i % (16 * RS);
          const int n = r / RS;
          buf(t, P)[r] = flag[n] ? buf(t, F)[r] : buf(t, U)[r];
        }
        for (int i = threadIdx.x; i < T * 16; i += nthr) {
          const int t = i / 16, n = i % 16;
          ebuf(t, P)[n] = flag[n] ? ebuf(t, F)[n] : ebuf(t, U)[n];
        }
        __syncthreads();
        pos = f + 1;
      }
    }
  }

  // write back
  for (int i = threadIdx.x; i < 16 * a.nw; i += nthr) {
    const int n = i / a.nw, wd = i % a.nw;
    if (a.mode == 1 && w0 + n < a.W) a.spins[(size_t)(w0 + n) * a.nw + wd] = sp[i];
  }
  if (threadIdx.x < 16 && w0 + threadIdx.x < a.W) {
    const int n = threadIdx.x, w = w0 + n;
    const bool ok = stat[n] == 0;
    if (a.logabs) a.logabs[w] = ok ? lab[n] : NAN;
    if (a.sign) a.sign[w] = ok ? (int8_t)sgn[n] : 0;
    if (a.accepts && a.mode == 1) a.accepts[w] += acc[n];
    if (a.status) a.status[w] = stat[n];
  }
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

__global__ void __launch_bounds__(256) reduce_kernel(int n, const double* x, double* out) {
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

}  // namespace rttk
