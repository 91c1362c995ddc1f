// Learned multi-spin proposal on gfx950: a 3-layer 3x3 convolutional
// network (32 channels, SiLU, periodic padding) with a 1x1 head giving, per
// site, one centre logit and eight size logits.  A move flips the first k
// sites of a fixed spiral around a sampled centre; the Metropolis-Hastings
// ratio uses the exact proposal probability of the flipped set in both
// directions, so the chain samples |psi|^2 whatever the weights are.
//
// One block of 256 threads per configuration, one thread per lattice site
// (N <= 256).  Weights are read with uniform addresses (scalar loads);
// activations live in LDS as [channel][site].
#pragma once
#include "rtt_device.hpp"

namespace rttk {

constexpr int kNetC = 32;
constexpr int kNetParams = 19113;
// offsets of the flattened parameters: W1, b1, W2, b2, W3, b3, Wh, bh
constexpr int oW1 = 0, ob1 = 288, oW2 = 320, ob2 = 9536, oW3 = 9568, ob3 = 18784, oWh = 18816,
              obh = 19104;
// spiral (dx, dy) around the centre
__constant__ const int kSpiralDx[8] = {0, 1, 1, 0, -1, -1, -1, 0};
__constant__ const int kSpiralDy[8] = {0, 0, 1, 1, 1, 0, -1, -1};

__device__ __forceinline__ float silu_f(float a) { return a / (1.f + __expf(-a)); }
__device__ __forceinline__ float silu_grad(float a) {
  const float s = 1.f / (1.f + __expf(-a));
  return s * (1.f + a * (1.f - s));
}

struct NetGeo {
  int Lx, Ly, N;
  int nb[9];  // neighbour (y + ky - 1, x + kx - 1) of this thread's site, tap = 3 ky + kx
  __device__ void init(int lx, int ly) {
    Lx = lx; Ly = ly; N = lx * ly;
    const int i = threadIdx.x < N ? threadIdx.x : 0;
    const int x = i % lx, y = i / lx;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int ky = t / 3, kx = t % 3;
      nb[t] = ((y + ky - 1 + ly) % ly) * lx + (x + kx - 1 + lx) % lx;
    }
  }
};

// One 3x3 layer for this thread's site: acc[co] = b[co] + sum W[co][ci][t] in(ci, nb[t]).
// in_act: whether the input buffer holds pre-activations (SiLU applied on read).
template <int CI>
__device__ __forceinline__ void conv_site(const float* __restrict__ W, const float* __restrict__ b,
                                          const float* in, bool in_act, const NetGeo& g,
                                          float (&acc)[kNetC]) {
#pragma unroll
  for (int co = 0; co < kNetC; ++co) acc[co] = b[co];
  for (int ci = 0; ci < CI; ++ci) {
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      float x = in[ci * g.N + g.nb[t]];
      if (in_act) x = silu_f(x);
#pragma unroll
      for (int co = 0; co < kNetC; ++co) acc[co] = fmaf(W[(co * CI + ci) * 9 + t], x, acc[co]);
    }
  }
}

// Forward pass of one configuration.  lds: z[N], then three [32][N] buffers
// A1, A2, A3 holding pre-activations, then o[9][N].  Returns pointer to o.
__device__ inline float* net_forward_block(const float* __restrict__ P, const uint64_t* spins,
                                           const NetGeo& g, float* lds) {
  const int N = g.N, i = threadIdx.x;
  const bool act = i < N;
  float* z = lds;
  float* A1 = z + 256;
  float* A2 = A1 + kNetC * N;
  float* A3 = A2 + kNetC * N;
  float* o = A3 + kNetC * N;
  if (act) z[i] = 1.f - 2.f * (float)spin_bit(spins, i);
  __syncthreads();
  float acc[kNetC];
  if (act) {
    conv_site<1>(P + oW1, P + ob1, z, false, g, acc);
#pragma unroll
    for (int co = 0; co < kNetC; ++co) A1[co * N + i] = acc[co];
  }
  __syncthreads();
  if (act) {
    conv_site<kNetC>(P + oW2, P + ob2, A1, true, g, acc);
#pragma unroll
    for (int co = 0; co < kNetC; ++co) A2[co * N + i] = acc[co];
  }
  __syncthreads();
  if (act) {
    conv_site<kNetC>(P + oW3, P + ob3, A2, true, g, acc);
#pragma unroll
    for (int co = 0; co < kNetC; ++co) A3[co * N + i] = acc[co];
  }
  __syncthreads();
  if (act) {
    float h[kNetC];
#pragma unroll
    for (int c = 0; c < kNetC; ++c) h[c] = silu_f(A3[c * N + i]);
    for (int k = 0; k < 9; ++k) {
      float s = P[obh + k];
#pragma unroll
      for (int c = 0; c < kNetC; ++c) s = fmaf(P[oWh + k * kNetC + c], h[c], s);
      o[k * N + i] = s;
    }
  }
  __syncthreads();
  return o;
}

// LDS of the scalar forward (training kernel): z, A1..A3, o, log-probs, scratch
__host__ __device__ inline size_t net_lds_bytes(int N) { return (size_t)(280 + 115 * N) * 4; }

// ---------------------------------------------------------------- matrix-core forward
// The two 32 -> 32 channel 3x3 layers as implicit GEMMs on the BF16 matrix
// cores: out^T[co][site] = sum over taps t and input channels ci of
// W[co][ci][t] h[ci][nb(site, t)], one 16 (channels) x 16 (sites) tile per
// matrix op sequence, K = 32 input channels per tap.  The weights are BF16
// values already; each activation enters as three BF16 parts hi + mid + lo
// (their sum equals it to about 2^-26 relative, finer than FP32 rounding),
// so with FP32 accumulation the layer keeps FP32 accuracy.  Activations are
// kept in LDS site-major, [site][channel], one plane per part.
// Packed weights: [layer 2, 3][tap][co][ci] BF16, written from the
// inference copy by net_pack_kernel.
constexpr int kNetPacked = 2 * 9 * kNetC * kNetC;

__global__ void net_pack_kernel(const float* infer, uint16_t* wpk) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNetPacked) return;
  const int layer = p / (9 * kNetC * kNetC), r = p % (9 * kNetC * kNetC);
  const int t = r / (kNetC * kNetC), co = (r / kNetC) % kNetC, ci = r % kNetC;
  const float w = infer[(layer == 0 ? oW2 : oW3) + (co * kNetC + ci) * 9 + t];
  wpk[p] = f32_to_bf16_rne(w);  // exact: the inference weights are BF16 values
}

__device__ __forceinline__ void split3_bf16(float x, uint16_t& h, uint16_t& m, uint16_t& l) {
  const __bf16 xh = (__bf16)x;
  const float r1 = x - (float)xh;
  const __bf16 xm = (__bf16)r1;
  const __bf16 xl = (__bf16)(r1 - (float)xm);
  h = __builtin_bit_cast(uint16_t, xh);
  m = __builtin_bit_cast(uint16_t, xm);
  l = __builtin_bit_cast(uint16_t, xl);
}

// sites padded to whole 16-site tiles
__host__ __device__ inline int net_padded(int N) { return (N + 15) / 16 * 16; }
// LDS (floats) of the matrix-core forward kernels: z[256], two activation
// buffers of three [NP][32] BF16 planes (the first later holds SiLU(a3) as
// [32][N] floats), o[9][N], then the log-probability area of the proposal
// kernels (lc[N] doubles, lk[8][N], reduction scratch, move, flip set)
__host__ __device__ inline size_t net_fwd_lds_bytes(int N) {
  return (size_t)(280 + 96 * net_padded(N) + 19 * N) * 4;
}

// One 32 -> 32 layer: input planes in (SiLU'd activations, split), output
// SiLU(a) either split into the planes out, or as FP32 [32][N] into h3.
__device__ __forceinline__ void net_conv_mfma(const uint16_t* __restrict__ wl, const float* __restrict__ bias,
                                              const uint16_t* in, uint16_t* out, float* h3, const NetGeo& g,
                                              int NP) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gq = lane >> 4, m = lane & 15;
  const int ct = wave >> 1;  // output channel tile of this wave
  const int N = g.N;
  bf16x8 wa[9];
#pragma unroll
  for (int t = 0; t < 9; ++t)
    wa[t] = *reinterpret_cast<const bf16x8*>(wl + ((size_t)t * kNetC + ct * 16 + m) * kNetC + 8 * gq);
  float bv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) bv[i] = bias[ct * 16 + 4 * gq + i];
  const size_t plane = (size_t)NP * kNetC;
  for (int st = wave & 1; st < NP / 16; st += 2) {
    const int site = st * 16 + m;
    const int sc = site < N ? site : 0;
    const int x = sc % g.Lx, y = sc / g.Lx;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
      yy += yy < 0 ? g.Ly : 0;
      yy -= yy >= g.Ly ? g.Ly : 0;
      xx += xx < 0 ? g.Lx : 0;
      xx -= xx >= g.Lx ? g.Lx : 0;
      const uint16_t* row = in + (size_t)(yy * g.Lx + xx) * kNetC + 8 * gq;
      const bf16x8 bl = *reinterpret_cast<const bf16x8*>(row + 2 * plane);
      const bf16x8 bm = *reinterpret_cast<const bf16x8*>(row + plane);
      const bf16x8 bh = *reinterpret_cast<const bf16x8*>(row);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t], bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t], bm, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t], bh, acc, 0, 0, 0);
    }
    if (site < N) {  // lane holds channels ct*16 + 4gq .. +3 of this site
      const int c0 = ct * 16 + 4 * gq;
      if (h3) {
#pragma unroll
        for (int i = 0; i < 4; ++i) h3[(c0 + i) * N + site] = silu_f(acc[i] + bv[i]);
      } else {
        uint16_t ph[4], pm[4], pl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) split3_bf16(silu_f(acc[i] + bv[i]), ph[i], pm[i], pl[i]);
        uint16_t* o = out + (size_t)site * kNetC + c0;
        *reinterpret_cast<uint2*>(o) = make_uint2(ph[0] | (uint32_t)ph[1] << 16, ph[2] | (uint32_t)ph[3] << 16);
        *reinterpret_cast<uint2*>(o + plane) =
            make_uint2(pm[0] | (uint32_t)pm[1] << 16, pm[2] | (uint32_t)pm[3] << 16);
        *reinterpret_cast<uint2*>(o + 2 * plane) =
            make_uint2(pl[0] | (uint32_t)pl[1] << 16, pl[2] | (uint32_t)pl[3] << 16);
      }
    }
  }
}

// Forward pass of one configuration with the layers above (256 threads:
// layer 1 and the head one thread per site, the two middle layers on the
// matrix cores).  Returns o[9][N] in LDS.
__device__ inline float* net_forward_mfma(const float* __restrict__ P, const uint16_t* __restrict__ wpk,
                                          const uint64_t* spins, const NetGeo& g, float* lds) {
  const int N = g.N, i = threadIdx.x, NP = net_padded(N);
  const bool act = i < N;
  float* z = lds;
  uint16_t* S0 = reinterpret_cast<uint16_t*>(lds + 256);
  uint16_t* S1 = S0 + 3 * NP * kNetC;
  float* H3 = reinterpret_cast<float*>(S0);  // S0 is free once layer 2 has run
  float* o = reinterpret_cast<float*>(S1 + 3 * NP * kNetC);
  if (act) z[i] = 1.f - 2.f * (float)spin_bit(spins, i);
  __syncthreads();
  if (act) {
    float acc[kNetC];
    conv_site<1>(P + oW1, P + ob1, z, false, g, acc);
    const size_t plane = (size_t)NP * kNetC;
#pragma unroll
    for (int c = 0; c < kNetC; c += 2) {
      uint16_t h0, m0, l0, h1, m1, l1;
      split3_bf16(silu_f(acc[c]), h0, m0, l0);
      split3_bf16(silu_f(acc[c + 1]), h1, m1, l1);
      uint32_t* row = reinterpret_cast<uint32_t*>(S0 + (size_t)i * kNetC + c);
      row[0] = h0 | (uint32_t)h1 << 16;
      row[plane / 2] = m0 | (uint32_t)m1 << 16;
      row[plane] = l0 | (uint32_t)l1 << 16;
    }
  }
  __syncthreads();
  net_conv_mfma(wpk, P + ob2, S0, S1, nullptr, g, NP);
  __syncthreads();
  net_conv_mfma(wpk + 9 * kNetC * kNetC, P + ob3, S1, nullptr, H3, g, NP);
  __syncthreads();
  if (act) {
    float h[kNetC];
#pragma unroll
    for (int c = 0; c < kNetC; ++c) h[c] = H3[c * N + i];
    for (int k = 0; k < 9; ++k) {
      float s = P[obh + k];
#pragma unroll
      for (int c = 0; c < kNetC; ++c) s = fmaf(P[oWh + k * kNetC + c], h[c], s);
      o[k * N + i] = s;
    }
  }
  __syncthreads();
  return o;
}

// block-wide reductions (256 threads)
__device__ inline double block_sum_d(double x, double* sh) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
  __syncthreads();
  const double r = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return r;
}
__device__ inline float block_max_f(float x, float* sh) {
  for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
  __syncthreads();
  const float r = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
  __syncthreads();
  return r;
}

// log-softmax of the centre logits over sites (block) and of this thread's
// eight size logits; writes lc[i] (log p(c = i)) and lk[8][i] into LDS.
__device__ inline void net_logprobs(const float* o, const NetGeo& g, double* lc, float* lk, double* shd,
                                    float* shf) {
  const int N = g.N, i = threadIdx.x;
  const bool act = i < N;
  const float m = block_max_f(act ? o[i] : -INFINITY, shf);
  const double se = block_sum_d(act ? exp((double)o[i] - (double)m) : 0.0, shd);
  const double lse = (double)m + log(se);
  if (act) {
    lc[i] = (double)o[i] - lse;
    float mk = -INFINITY;
    for (int k = 0; k < 8; ++k) mk = fmaxf(mk, o[(k + 1) * N + i]);
    double s = 0.0;
    for (int k = 0; k < 8; ++k) s += exp((double)o[(k + 1) * N + i] - (double)mk);
    const double l = (double)mk + log(s);
    for (int k = 0; k < 8; ++k) lk[k * N + i] = (float)((double)o[(k + 1) * N + i] - l);
  }
  __syncthreads();
}

__device__ __forceinline__ int spiral_site(int c, int m, int Lx, int Ly) {
  const int x = c % Lx, y = c / Lx;
  return ((y + kSpiralDy[m] + Ly) % Ly) * Lx + (x + kSpiralDx[m] + Lx) % Lx;
}

// q(S|s) for the flip set S of move (c, k): sum of p(c') p(k|c') over the
// centres c' whose k-site spiral equals S (sets of different sizes differ).
__device__ inline double net_set_prob(const double* lc, const float* lk, const NetGeo& g, int c, int k,
                                      const uint64_t* target, double* shd) {
  const int i = threadIdx.x;
  double p = 0.0;
  if (i < g.N) {
    bool same = true;
    for (int m = 0; m < k; ++m) {
      const int s = spiral_site(i, m, g.Lx, g.Ly);
      same &= ((target[s >> 6] >> (s & 63)) & 1ull) != 0ull;
    }
    if (same) p = exp(lc[i] + (double)lk[(k - 1) * g.N + i]);
  }
  return block_sum_d(p, shd);
}

struct NetMoveArgs {
  const float* P;          // inference weights
  const uint16_t* wpk;     // the middle layers' weights packed for the matrix cores
  int Lx, Ly, nw, W;
  const uint64_t* spins;   // [W][nw] current
  uint64_t* prop;          // [W][nw] proposed (written by propose)
  int* moves;              // [W] c | k << 16
  double* lqf;             // [W] log q(S|s)
  double* lqr;             // [W] log q(S|s')
  uint64_t seed, rstream, step;
  float* out;              // [W][9][N] head outputs (forward only) or null
  uint64_t* before;        // [W][nw] copy of the state the move was proposed at, or null
};

// propose: forward at s, sample (c, k), write s' and log q(S|s)
__global__ void __launch_bounds__(256) net_propose_kernel(NetMoveArgs a) {
  extern __shared__ __align__(16) float lds[];
  NetGeo g;
  g.init(a.Lx, a.Ly);
  const int w = blockIdx.x, N = g.N;
  const uint64_t* sw = a.spins + (size_t)w * a.nw;
  float* o = net_forward_mfma(a.P, a.wpk, sw, g, lds);
  double* lc = reinterpret_cast<double*>(o + 9 * N + (N & 1));
  float* lk = reinterpret_cast<float*>(lc + N);
  double* shd = reinterpret_cast<double*>(lk + 8 * N + ((8 * N) & 1));
  float* shf = reinterpret_cast<float*>(shd + 4);
  int* mv = reinterpret_cast<int*>(shf + 4);
  uint64_t* tgt = reinterpret_cast<uint64_t*>(mv + 2);
  net_logprobs(o, g, lc, lk, shd, shf);
  // inverse-CDF draw of the centre: inclusive prefix sums of p(c = i) over
  // the sites (FP64 block scan in site order), c = the first site whose sum
  // exceeds uc (the last site if none does)
  {
    const int i = threadIdx.x, lane = i & 63, wv = i >> 6;
    const double uc = philox_uniform(a.seed, a.rstream, (uint64_t)w, a.step, (1ull << 32) + 0);
    double cum = i < N ? exp(lc[i]) : 0.0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double y = __shfl_up(cum, o);
      if (lane >= o) cum += y;
    }
    if (lane == 63) shd[wv] = cum;
    __syncthreads();
    for (int q = 0; q < wv; ++q) cum += shd[q];
    int cand = (i < N && cum > uc) ? i : N - 1;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cand = min(cand, __shfl_xor(cand, o));
    int* shi = reinterpret_cast<int*>(shf);
    __syncthreads();
    if (lane == 0) shi[wv] = cand;
    __syncthreads();
    if (i == 0) mv[0] = min(min(shi[0], shi[1]), min(shi[2], shi[3]));
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double uk = philox_uniform(a.seed, a.rstream, (uint64_t)w, a.step, (1ull << 32) + 1);
    const int c = mv[0];
    double cum = 0.0;
    int k = 8;
    for (int m = 0; m < 8; ++m) {
      cum += exp((double)lk[m * N + c]);
      if (cum > uk) { k = m + 1; break; }
    }
    mv[0] = c;
    mv[1] = k;
    for (int q = 0; q < a.nw; ++q) tgt[q] = 0ull;
    for (int m = 0; m < k; ++m) {
      const int s = spiral_site(c, m, a.Lx, a.Ly);
      tgt[s >> 6] |= 1ull << (s & 63);
    }
  }
  __syncthreads();
  const int c = mv[0], k = mv[1];
  const double q = net_set_prob(lc, lk, g, c, k, tgt, shd);
  if (threadIdx.x == 0) {
    a.moves[w] = c | (k << 16);
    a.lqf[w] = log(q);
  }
  if (threadIdx.x < a.nw) {
    a.prop[(size_t)w * a.nw + threadIdx.x] = sw[threadIdx.x] ^ tgt[threadIdx.x];
    if (a.before) a.before[(size_t)w * a.nw + threadIdx.x] = sw[threadIdx.x];
  }
}

// reverse: forward at s', log q(S|s') for the same set
__global__ void __launch_bounds__(256) net_reverse_kernel(NetMoveArgs a) {
  extern __shared__ __align__(16) float lds[];
  NetGeo g;
  g.init(a.Lx, a.Ly);
  const int w = blockIdx.x, N = g.N;
  float* o = net_forward_mfma(a.P, a.wpk, a.prop + (size_t)w * a.nw, g, lds);
  double* lc = reinterpret_cast<double*>(o + 9 * N + (N & 1));
  float* lk = reinterpret_cast<float*>(lc + N);
  double* shd = reinterpret_cast<double*>(lk + 8 * N + ((8 * N) & 1));
  float* shf = reinterpret_cast<float*>(shd + 4);
  int* mv = reinterpret_cast<int*>(shf + 4);
  uint64_t* tgt = reinterpret_cast<uint64_t*>(mv + 2);
  net_logprobs(o, g, lc, lk, shd, shf);
  const int c = a.moves[w] & 0xffff, k = a.moves[w] >> 16;
  if (threadIdx.x == 0) {
    for (int q = 0; q < a.nw; ++q) tgt[q] = 0ull;
    for (int m = 0; m < k; ++m) {
      const int s = spiral_site(c, m, a.Lx, a.Ly);
      tgt[s >> 6] |= 1ull << (s & 63);
    }
  }
  __syncthreads();
  const double q = net_set_prob(lc, lk, g, c, k, tgt, shd);
  if (threadIdx.x == 0) a.lqr[w] = log(q);
}

// forward only: head outputs to global memory
__global__ void __launch_bounds__(256) net_forward_kernel(NetMoveArgs a) {
  extern __shared__ __align__(16) float lds[];
  NetGeo g;
  g.init(a.Lx, a.Ly);
  const int w = blockIdx.x, N = g.N;
  const float* o = net_forward_mfma(a.P, a.wpk, a.spins + (size_t)w * a.nw, g, lds);
  for (int i = threadIdx.x; i < 9 * N; i += 256) a.out[(size_t)w * 9 * N + i] = o[i];
}

// acceptance (one thread per walker): u < |psi'/psi|^2 q(S|s') / q(S|s)
struct NetAcceptArgs {
  int W, nw;
  uint64_t* spins; const uint64_t* prop;
  double* logabs; int8_t* sign;
  const double* la_new; const int8_t* sg_new; const int32_t* st_new;
  const double* lqf; const double* lqr;
  const int* moves; float* accept_prob;
  uint32_t* accepts; int32_t* status;
  uint64_t seed, rstream, step;
};
__global__ void net_accept_kernel(NetAcceptArgs a) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= a.W) return;
  const bool ok_old = isfinite(a.logabs[w]) && a.sign[w] != 0;
  const bool ok_new = a.st_new[w] == 0;
  double A = 0.0;
  if (ok_old && ok_new) A = exp(2.0 * (a.la_new[w] - a.logabs[w]) + a.lqr[w] - a.lqf[w]);
  const double u = philox_uniform(a.seed, a.rstream, (uint64_t)w, a.step, (1ull << 32) + 2);
  const bool acc = ok_old && ok_new && u < A;
  if (a.accept_prob) a.accept_prob[w] = (float)fmin(1.0, A);
  if (acc) {
    for (int q = 0; q < a.nw; ++q) a.spins[(size_t)w * a.nw + q] = a.prop[(size_t)w * a.nw + q];
    a.logabs[w] = a.la_new[w];
    a.sign[w] = a.sg_new[w];
    if (a.accepts) a.accepts[w] += 1;
  }
  if (a.status) a.status[w] = ok_old ? 0 : -5;
}

// ---------------------------------------------------------------- training
struct NetGradArgs {
  const float* P;          // weights the forward pass uses
  int Lx, Ly, nw, B;
  const uint64_t* spins;   // [B][nw] states s_b
  const int* moves;        // [B] c | k << 16 sampled at s_b
  const float* accept_prob;// [B]
  const double* baseline;  // device scalar
  float* partial;          // [B][kNetParams] per-sample gradients
};

// Gradient of coef_b log q(c_b, k_b | s_b), coef_b = -(a_b k_b - baseline) / B.
__global__ void __launch_bounds__(256) net_grad_kernel(NetGradArgs a) {
  extern __shared__ __align__(16) float lds[];
  NetGeo g;
  g.init(a.Lx, a.Ly);
  const int b = blockIdx.x, N = g.N, i = threadIdx.x;
  const bool act = i < N;
  float* o = net_forward_block(a.P, a.spins + (size_t)b * a.nw, g, lds);
  float* z = lds;
  float* A1 = z + 256;
  float* A2 = A1 + kNetC * N;
  float* A3 = A2 + kNetC * N;
  float* G = o + 9 * N;                       // [32][N] gradient buffer
  double* lc = reinterpret_cast<double*>(G + kNetC * N + (N & 1));
  float* lk = reinterpret_cast<float*>(lc + N);
  double* shd = reinterpret_cast<double*>(lk + 8 * N + ((8 * N) & 1));
  float* shf = reinterpret_cast<float*>(shd + 4);
  net_logprobs(o, g, lc, lk, shd, shf);
  const int c = a.moves[b] & 0xffff, k = a.moves[b] >> 16;
  const double coef = -((double)a.accept_prob[b] * k - *a.baseline) / a.B;
  float* out = a.partial + (size_t)b * kNetParams;
  // d loss / d o, written over o: channel 0 at every site, size channels at c
  if (act) {
    o[i] = (float)(coef * ((i == c ? 1.0 : 0.0) - exp(lc[i])));
    for (int m = 0; m < 8; ++m)
      o[(m + 1) * N + i] = (i == c) ? (float)(coef * ((m + 1 == k ? 1.0 : 0.0) - exp((double)lk[m * N + i]))) : 0.f;
  }
  __syncthreads();
  // head: dWh[k][ch] = sum_i do[k][i] h3[ch][i], dbh[k] = sum_i do[k][i]
  for (int p = i; p < 9 * kNetC + 9; p += 256) {
    float s = 0.f;
    if (p < 9 * kNetC) {
      const int kk = p / kNetC, ch = p % kNetC;
      for (int j = 0; j < N; ++j) s = fmaf(o[kk * N + j], silu_f(A3[ch * N + j]), s);
      out[oWh + p] = s;
    } else {
      const int kk = p - 9 * kNetC;
      for (int j = 0; j < N; ++j) s += o[kk * N + j];
      out[obh + kk] = s;
    }
  }
  // dh3 -> G, then da3 = dh3 * SiLU'(a3)
  if (act) {
    for (int ch = 0; ch < kNetC; ++ch) {
      float s = 0.f;
      for (int kk = 0; kk < 9; ++kk) s = fmaf(a.P[oWh + kk * kNetC + ch], o[kk * N + i], s);
      G[ch * N + i] = s * silu_grad(A3[ch * N + i]);
    }
  }
  __syncthreads();
  // layer 3 (input h2 = SiLU(A2)) and layer 2 (input h1 = SiLU(A1)):
  // dW[co][ci][t] = sum_i da[co][i] h[ci][nb(i, t)], db[co] = sum_i da[co][i],
  // dh[ci][j] = sum_{co,t} W[co][ci][t] da[co][nb(j, 8 - t)]
  auto conv_back = [&](const float* __restrict__ Wl, int oW, int ob, const float* da, const float* ain,
                       float* dh_out) {
    for (int p = i; p < kNetC * 9; p += 256) {
      const int ci = p / 9, t = p % 9;
      float acc[kNetC];
#pragma unroll
      for (int co = 0; co < kNetC; ++co) acc[co] = 0.f;
      for (int j = 0; j < N; ++j) {
        // the site whose tap-t neighbour is read at j's position: input at nb(j, t)
        const int x = j % g.Lx, y = j / g.Lx;
        const int nbj = ((y + t / 3 - 1 + g.Ly) % g.Ly) * g.Lx + (x + t % 3 - 1 + g.Lx) % g.Lx;
        const float hv = silu_f(ain[ci * N + nbj]);
#pragma unroll
        for (int co = 0; co < kNetC; ++co) acc[co] = fmaf(da[co * N + j], hv, acc[co]);
      }
#pragma unroll
      for (int co = 0; co < kNetC; ++co) out[oW + (co * kNetC + ci) * 9 + t] = acc[co];
    }
    for (int co = i; co < kNetC; co += 256) {
      float s = 0.f;
      for (int j = 0; j < N; ++j) s += da[co * N + j];
      out[ob + co] = s;
    }
    float acc[kNetC];
#pragma unroll
    for (int ci = 0; ci < kNetC; ++ci) acc[ci] = 0.f;
    if (act) {
      for (int co = 0; co < kNetC; ++co)
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          const float d = da[co * N + g.nb[8 - t]];
#pragma unroll
          for (int ci = 0; ci < kNetC; ++ci) acc[ci] = fmaf(Wl[(co * kNetC + ci) * 9 + t], d, acc[ci]);
        }
      // dh_out is none of the buffers read above
#pragma unroll
      for (int ci = 0; ci < kNetC; ++ci) dh_out[ci * N + i] = acc[ci] * silu_grad(ain[ci * N + i]);
    }
    __syncthreads();
  };
  conv_back(a.P + oW3, oW3, ob3, G, A2, A3);   // A3 is free: da2 goes there
  conv_back(a.P + oW2, oW2, ob2, A3, A1, G);   // da1 goes to G
  // layer 1: input z, one channel
  for (int p = i; p < kNetC * 9; p += 256) {
    const int co = p / 9, t = p % 9;
    float s = 0.f;
    for (int j = 0; j < N; ++j) {
      const int x = j % g.Lx, y = j / g.Lx;
      const int nbj = ((y + t / 3 - 1 + g.Ly) % g.Ly) * g.Lx + (x + t % 3 - 1 + g.Lx) % g.Lx;
      s = fmaf(G[co * N + j], z[nbj], s);
    }
    out[oW1 + co * 9 + t] = s;
  }
  for (int co = i; co < kNetC; co += 256) {
    float s = 0.f;
    for (int j = 0; j < N; ++j) s += G[co * N + j];
    out[ob1 + co] = s;
  }
}

__host__ __device__ inline size_t net_grad_lds_bytes(int N) { return (size_t)(280 + 147 * N) * 4; }

// Sum over samples in two fixed-order stages: slice y of S adds its share
// of the samples, then net_reduce_kernel adds the S slices.
__global__ void net_reduce_slices_kernel(const float* partial, int B, int S, float* out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (p >= kNetParams) return;
  const int b0 = (int)((long long)B * y / S), b1 = (int)((long long)B * (y + 1) / S);
  float s = 0.f;
  for (int b = b0; b < b1; ++b) s += partial[(size_t)b * kNetParams + p];
  out[(size_t)y * kNetParams + p] = s;
}

// grad[p] = sum_b partial[b][p] (fixed order); baseline <- 0.9 baseline + 0.1 mean(a k)
__global__ void net_reduce_kernel(const float* partial, int B, float* grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNetParams) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += partial[(size_t)b * kNetParams + p];
  grad[p] = s;
}
__global__ void net_baseline_kernel(const float* accept_prob, const int* moves, int B, double* baseline) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int b = threadIdx.x; b < B; b += 256) s += (double)accept_prob[b] * (moves[b] >> 16);
  s = block_sum_d(s, sh);
  if (threadIdx.x == 0) *baseline = 0.9 * *baseline + 0.1 * (s / B);
}

// Adam on the FP32 master weights; the inference copy is rounded to BF16
__global__ void net_adam_kernel(float* master, float* infer, float* m, float* v, const float* grad,
                                float lr, float b1, float b2, float eps, int t) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNetParams) return;
  const float gp = grad[p];
  const float mp = b1 * m[p] + (1.f - b1) * gp;
  const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  const float mh = mp / (1.f - powf(b1, (float)t));
  const float vh = vp / (1.f - powf(b2, (float)t));
  const float w = master[p] - lr * mh / (sqrtf(vh) + eps);
  master[p] = w;
  infer[p] = bf16_to_f32(f32_to_bf16_rne(w));
}

}  // namespace rttk
