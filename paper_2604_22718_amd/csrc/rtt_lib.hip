// Host side of the RTT library: argument checks, core quantisation and
// packing, contraction schedules, workspace and kernel launches.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/rtt.h"
#include "rtt_kernels.hpp"
#include "rtt_narrow.hpp"
#include "rtt_net.hpp"
#include "rtt_tt.hpp"

namespace {

thread_local std::string g_err;

rtt_status fail(rtt_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPX(call)                                                                   \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(e_ == hipErrorOutOfMemory ? RTT_E_OOM : RTT_E_HIP, "%s: %s (%s:%d)", \
                  #call, hipGetErrorString(e_), __FILE__, __LINE__);                 \
  } while (0)

constexpr size_t kLdsLimit = 160 * 1024;
constexpr int kPassOccupancy = 2;  // pass blocks per CU worth trading extra row groups for

// ------------------------------------------------------------------ quantisation
float to_f32(double x) { return (float)x; }

uint16_t bf16_bits_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
double bf16_value(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

// OCP e4m3 ("fn"): round-to-nearest-even of a float already divided by the
// power-of-two scale, clamped to +-448 first.  Returns the decoded value.
double e4m3_round(float f) {
  double a = fabs((double)f);
  const double sg = f < 0 ? -1.0 : 1.0;
  if (a > 448.0) a = 448.0;
  const double min_normal = ldexp(1.0, -6);
  double q;
  if (a < min_normal) {
    q = nearbyint(a * 512.0) / 512.0;  // subnormal spacing 2^-9
  } else {
    int ex = 0;
    frexp(a, &ex);                     // a = m 2^ex, m in [0.5, 1)
    const double step = ldexp(1.0, ex - 1 - 3);  // 3 mantissa bits
    q = nearbyint(a / step) * step;
  }
  return sg * q;
}

// OCP e4m3 byte of a value that e4m3 represents exactly (|v| <= 448)
uint8_t e4m3_code(double v) {
  const uint8_t sg = v < 0 ? 0x80 : 0x00;
  const double a = fabs(v);
  if (a == 0.0) return sg;
  if (a < ldexp(1.0, -6)) return sg | (uint8_t)lrint(a * 512.0);  // subnormal: m * 2^-9
  int ex = 0;
  const double f = frexp(a, &ex);                               // a = f 2^ex, f in [0.5, 1)
  return sg | (uint8_t)((ex + 6) << 3) | (uint8_t)lrint((2.0 * f - 1.0) * 8.0);
}
double e4m3_decode(uint8_t b) {
  const int e = (b >> 3) & 15, m = b & 7;
  const double v = e == 0 ? m * ldexp(1.0, -9) : ldexp(1.0 + m / 8.0, e - 7);
  return (b & 0x80) ? -v : v;
}

int fp8_scale_exponent(const double* c, size_t n) {
  double amax = 0.0;
  for (size_t i = 0; i < n; ++i) amax = std::max(amax, fabs(c[i]));
  if (amax == 0.0) return 0;
  return (int)ceil(log2(amax / 448.0));
}

int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

struct Sched {
  std::vector<int> fwd, bwd;     // int4 entries of every row group, concatenated
  std::vector<int> fgs, bgs;     // int2 per group: (first entry, number of entries)
  std::vector<int> fslot, bslot, grp;
  int cut = 0, nslot = 16, ng = 1;
  long cost = 0;
};

// Forward steps over positions [0, c), backward steps over [c, L) from the
// right.  Spins are dealt round-robin, in order of first position, into ng
// row groups; one pass of group g carries the base vector and one vector
// per spin of g, spawned at the spin's first position (forward) or last
// position (backward) on its side of the cut.  At positions of spins of
// other groups every vector uses the walker's slice (no odd row, w = -1).
Sched build_sched(const std::vector<int>& pi, int N, int L, int c, int ng) {
  Sched s;
  s.cut = c;
  s.ng = ng;
  s.fslot.assign(N, 0);
  s.bslot.assign(N, 0);
  s.grp.assign(N, 0);
  std::vector<int> first(N, -1);
  for (int k = 0; k < L; ++k)
    if (first[pi[k]] < 0) first[pi[k]] = k;
  std::vector<int> order;
  for (int k = 0; k < L; ++k)
    if (first[pi[k]] == k) order.push_back(pi[k]);
  for (int r = 0; r < (int)order.size(); ++r) s.grp[order[r]] = r % ng;
  int nmax = 1;
  for (int g = 0; g < ng; ++g) {
    std::vector<int> fs(N, -1), bs(N, -1);
    const int f0 = (int)s.fwd.size() / 4, b0 = (int)s.bwd.size() / 4;
    int nf = 1;
    for (int k = 0; k < c; ++k) {
      const int q = pi[k];
      int odd = -1;
      if (s.grp[q] == g) {
        if (fs[q] < 0) { fs[q] = nf++; odd = 0 | (fs[q] << 16); }
        else odd = fs[q] | (fs[q] << 16);
      }
      s.fwd.insert(s.fwd.end(), {k, q, nf, odd});
      s.cost += (nf + 15) / 16;
    }
    int nb = 1;
    for (int k = L - 1; k >= c; --k) {
      const int q = pi[k];
      int odd = -1;
      if (s.grp[q] == g) {
        if (bs[q] < 0) { bs[q] = nb++; odd = 0 | (bs[q] << 16); }
        else odd = bs[q] | (bs[q] << 16);
      }
      s.bwd.insert(s.bwd.end(), {k, q, nb, odd});
      s.cost += (nb + 15) / 16;
    }
    s.fgs.insert(s.fgs.end(), {f0, c});
    s.bgs.insert(s.bgs.end(), {b0, L - c});
    for (int j = 0; j < N; ++j)
      if (s.grp[j] == g) {
        s.fslot[j] = fs[j] < 0 ? 0 : fs[j];
        s.bslot[j] = bs[j] < 0 ? 0 : bs[j];
      }
    nmax = std::max(nmax, std::max(nf, nb));
  }
  s.nslot = (nmax + 15) / 16 * 16;
  return s;
}

int rttk_wpw(int chi) { return chi >= 64 ? 4 : chi / 16; }

// the passes of rttk::pass_wide_form run the K-outer form (rows in place
// when so built, and at most kPassWideTiles row tiles per walker)
bool pass_wide(int dtype, int chi) {
  return PASS_W_ENABLE && ((dtype == RTT_FP8_E4M3 && (chi == 256 || (PASS_W_128 && chi == 128))) ||
                           (dtype == RTT_BF16 && PASS_W_128 && chi == 128));
}
int pass_max_slots(int dtype, int chi) { return pass_wide(dtype, chi) ? 16 * rttk::kPassWideTiles : 1 << 30; }

size_t pass_lds_bytes(int chi, int nslot, int nw, int dtype) {
  const int wpw = chi >= 64 ? 4 : chi / 16;
  const int wpb = 4 / wpw;
  const size_t rs = chi + 4;
  const int nb = (pass_wide(dtype, chi) && rttk::kPassWideInPlace) ? 1 : 2;  // row buffers
  return (size_t)wpb * (nb * nslot * rs * 4 + nb * nslot * 4 + nw * 8);
}

size_t chain_lds_bytes(int chi, int T, int L, int nw, int n_spins, int cg = 1) {
  return (size_t)rttk::ChainLayout(chi, T, (L + 63) / 64, nw, cg, 0, n_spins).total;
}

}  // namespace

struct rtt_s {
  int N = 0, L = 0, chi = 0, dtype = 0, T = 1, nw = 0, device = 0;
  std::vector<int> pi, bond;
  std::vector<double> coeffs;
  std::vector<std::vector<double>> qcores;  // quantised values, rtt_create layout, per term
  std::vector<std::vector<int>> fp8e;       // [T][L] FP8 scale exponents (FP8 cores only)
  std::vector<int> core_exp;                // [T][L] power-of-two scale of each stored core
  std::vector<int> cesum;                   // [T][L+1] prefix sums of core_exp
  std::vector<uint64_t> rmask;              // [N][LW] replica positions of each spin
  Sched sched;
  std::vector<int> order, first;
  // device
  void* d_fwd = nullptr;      // [T][L][2][chi*chi] transposed fragments
  void* d_bwd = nullptr;      // [T][L][2][chi*chi]
  int* d_cexp = nullptr;
  int* d_cesum = nullptr;
  uint64_t* d_rmask = nullptr;
  int4* d_sf = nullptr;
  int4* d_sb = nullptr;
  int* d_fslot = nullptr;
  int* d_bslot = nullptr;
  int* d_grp = nullptr;
  int2* d_fgs = nullptr;
  int2* d_bgs = nullptr;
  int* d_pi = nullptr;
  int* d_order = nullptr;
  int* d_first = nullptr;
  double* d_coeffs = nullptr;
  // narrow-bond path (every bond <= 4): C x C slices, prescaled, zero padded
  int narrow = 0;             // C = 2 or 4, 0 when the matrix-core path runs
  int chain_ck = 1;           // sweeps keep column checkpoints in LDS
  float* d_ncores = nullptr;  // [T][L][2][C][C]
  // workspace
  size_t ws_W = 0;
  float* d_u = nullptr;
  float* d_v = nullptr;
  int* d_ue = nullptr;
  int* d_ve = nullptr;
  float* d_ck = nullptr;      // global column checkpoints of the sequential sampler layout
  size_t ck_bytes = 0;
  // this state's amplitudes and local energies as a dual Monte Carlo target
  size_t mix_W = 0;
  double* d_mla = nullptr;
  int8_t* d_msg = nullptr;
  double* d_mel = nullptr;
  int32_t* d_mst = nullptr;
};

struct rtt_ham_s {
  int Lx = 0, Ly = 0, periodic = 0, nb = 0;
  double J = 0, h = 0;
  int2* d_bonds = nullptr;
};

namespace {

size_t elem_bytes(int dtype) { return dtype == RTT_F32 ? 4 : dtype == RTT_BF16 ? 2 : 1; }

// Pack one term: element (t, lane, e) of slice (k, b) in the forward layout
// is core[b][g*KPL + e][16t + m] (transposed), in the backward layout
// core[b][16t + m][g*KPL + e]; lane = 16 g + m, KPL = chi / 4.  Within the
// 64 * KPL elements of tile t the order is rttk::frag_offset's.  Elements are
// the quantised core divided by 2^core_exp: FP32 and BF16 values, or for FP8
// the e4m3 code c of the value c * 2^-9 (core_exp = FP8 scale + 9).
void pack_term(const rtt_s* h, int term, const std::vector<double>& q, std::vector<uint8_t>& fw,
               std::vector<uint8_t>& bw) {
  const int chi = h->chi, L = h->L, KPL = chi / 4;
  const size_t eb = elem_bytes(h->dtype);
  const size_t slice = (size_t)chi * chi;
  fw.assign((size_t)L * 2 * slice * eb, 0);
  bw.assign((size_t)L * 2 * slice * eb, 0);
  size_t off = 0;
  for (int k = 0; k < L; ++k) {
    const int a = h->bond[k], b = h->bond[k + 1];
    const int ce = h->core_exp[(size_t)term * L + k];
    std::vector<double> pad((size_t)2 * slice, 0.0);
    for (int s = 0; s < 2; ++s)
      for (int i = 0; i < a; ++i)
        for (int j = 0; j < b; ++j)
          pad[s * slice + (size_t)i * chi + j] = ldexp(q[off + ((size_t)s * a + i) * b + j], -ce);
    off += (size_t)2 * a * b;
    for (int s = 0; s < 2; ++s) {
      const size_t base = ((size_t)k * 2 + s) * slice;
      for (int t = 0; t < chi / 16; ++t)
        for (int lane = 0; lane < 64; ++lane)
          for (int e = 0; e < KPL; ++e) {
            const int g = lane >> 4, m = lane & 15;
            const size_t idx = base + (size_t)t * 64 * KPL + rttk::frag_offset(lane, e, rttk::frag_chunk((int)eb, KPL));
            const double vf = pad[s * slice + (size_t)(g * KPL + e) * chi + 16 * t + m];
            const double vb = pad[s * slice + (size_t)(16 * t + m) * chi + g * KPL + e];
            if (eb == 4) {
              const float ff = (float)vf, fb = (float)vb;
              memcpy(&fw[idx * 4], &ff, 4);
              memcpy(&bw[idx * 4], &fb, 4);
            } else if (eb == 1) {
              fw[idx] = e4m3_code(vf * 512.0);
              bw[idx] = e4m3_code(vb * 512.0);
              if (e4m3_decode(fw[idx]) != vf * 512.0 || e4m3_decode(bw[idx]) != vb * 512.0)
                throw std::runtime_error("FP8 packing: a core value is not an e4m3 code times its scale");
            } else {
              const uint16_t hf = bf16_bits_rne((float)vf), hb = bf16_bits_rne((float)vb);
              memcpy(&fw[idx * 2], &hf, 2);
              memcpy(&bw[idx * 2], &hb, 2);
            }
          }
    }
  }
}

rtt_status upload(void** dst, const void* src, size_t bytes) {
  HIPX(hipMalloc(dst, std::max<size_t>(bytes, 16)));
  if (bytes) HIPX(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
  return RTT_OK;
}

// Frees every device buffer of a handle; the caller has synchronised.  The
// workspace came from the stream-ordered allocator and goes back to it.
void free_dev(rtt_s* h) {
  void* ptrs[] = {h->d_grp, h->d_fgs, h->d_bgs, h->d_fwd, h->d_bwd, h->d_cexp, h->d_cesum, h->d_rmask, h->d_sf, h->d_sb, h->d_fslot, h->d_bslot,
                  h->d_pi, h->d_order, h->d_first, h->d_coeffs, h->d_ncores};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  void* ws[] = {h->d_u, h->d_v, h->d_ue, h->d_ve, h->d_mla, h->d_msg, h->d_mel, h->d_mst, h->d_ck};
  bool any = false;
  for (void* p : ws)
    if (p) { (void)hipFreeAsync(p, nullptr); any = true; }
  if (any) (void)hipDeviceSynchronize();
}

// Quantised copy of the cores (rtt_create layout) and, for FP8, the scale
// exponent of each position.
void quantise(int dtype, const std::vector<int>& bond, const double* cores, std::vector<double>& q,
              std::vector<int>& cexp) {
  const int L = (int)bond.size() - 1;
  size_t off = 0;
  q.clear();
  cexp.assign(L, 0);
  for (int k = 0; k < L; ++k) {
    const size_t n = (size_t)2 * bond[k] * bond[k + 1];
    const double* c = cores + off;
    if (dtype == RTT_F32) {
      for (size_t i = 0; i < n; ++i) q.push_back((double)to_f32(c[i]));
    } else if (dtype == RTT_BF16) {
      for (size_t i = 0; i < n; ++i) q.push_back(bf16_value(bf16_bits_rne((float)c[i])));
    } else {  // FP8 e4m3: value = code * 2^e, one scale per position
      const int e = fp8_scale_exponent(c, n);
      for (size_t i = 0; i < n; ++i) q.push_back(ldexp(e4m3_round((float)ldexp(c[i], -e)), e));
      cexp[k] = e;
    }
    off += n;
  }
}

// Every stored core is the quantised core times 2^-e_k, with e_k chosen so
// that its largest entry lies in [0.5, 1): exact, and it bounds the growth
// of a renormalised row to chi per step.  e_k is added back in the exponent
// bookkeeping of the kernels.  FP8 cores are stored as their codes, which the
// kernels read as code * 2^-9 (below 1 as well): e_k = FP8 scale + 9.
void prescale(rtt_s* h) {
  h->core_exp.assign((size_t)h->T * h->L, 0);
  h->cesum.assign((size_t)h->T * (h->L + 1), 0);
  for (int t = 0; t < h->T; ++t) {
    std::vector<double>& q = h->qcores[t];
    size_t off = 0;
    for (int k = 0; k < h->L; ++k) {
      const size_t n = (size_t)2 * h->bond[k] * h->bond[k + 1];
      double amax = 0.0;
      for (size_t i = 0; i < n; ++i) amax = std::max(amax, fabs(q[off + i]));
      int e = 0;
      if (h->dtype == RTT_FP8_E4M3) e = h->fp8e[t][k] + 9;
      else if (amax > 0.0) frexp(amax, &e);
      h->core_exp[(size_t)t * h->L + k] = e;
      h->cesum[(size_t)t * (h->L + 1) + k + 1] = h->cesum[(size_t)t * (h->L + 1) + k] + e;
      off += n;
    }
  }
}

size_t narrow_chain_lds(const rtt_s* h) { return (size_t)((h->L + 63) / 64 + h->nw) * 64 * 8; }

// Trains with every bond <= 4 also get C x C slices (C = 2 or 4) for the
// vector-ALU kernels, the same prescaled values as the packed fragments.
rtt_status setup_narrow(rtt_s* h) {
  int bmax = 1;
  for (int b : h->bond) bmax = std::max(bmax, b);
  h->narrow = 0;
  if (bmax > rttn::kNarrowMax || h->T > rttn::kMaxTermsN || narrow_chain_lds(h) > kLdsLimit) return RTT_OK;
  const char* off = getenv("RTT_NARROW");
  if (off && off[0] == '0') return RTT_OK;
  const int C = bmax <= 2 ? 2 : 4;
  std::vector<float> nc((size_t)h->T * h->L * 2 * C * C, 0.f);
  for (int t = 0; t < h->T; ++t) {
    const std::vector<double>& q = h->qcores[t];
    size_t off = 0;
    for (int k = 0; k < h->L; ++k) {
      const int ra = h->bond[k], rb = h->bond[k + 1];
      const int e = h->core_exp[(size_t)t * h->L + k];
      float* dst = nc.data() + ((size_t)t * h->L + k) * 2 * C * C;
      for (int sl = 0; sl < 2; ++sl)
        for (int r = 0; r < ra; ++r)
          for (int c = 0; c < rb; ++c)
            dst[sl * C * C + r * C + c] = (float)ldexp(q[off + ((size_t)sl * ra + r) * rb + c], -e);
      off += (size_t)2 * ra * rb;
    }
  }
  rtt_status st = upload((void**)&h->d_ncores, nc.data(), nc.size() * 4);
  if (st != RTT_OK) return st;
  h->narrow = C;
  return RTT_OK;
}

rtt_status finish_create(rtt_s* h) {
  prescale(h);
  const int LW = (h->L + 63) / 64;
  h->rmask.assign((size_t)h->N * LW, 0ull);
  for (int k = 0; k < h->L; ++k) h->rmask[(size_t)h->pi[k] * LW + k / 64] |= 1ull << (k % 64);
  // Schedules: over row-group counts and cut bonds whose rows fit on chip,
  // minimise matrix-core tiles divided by the pass blocks resident per CU
  // (counted up to kPassOccupancy: one block per CU leaves every latency
  // of the step exposed; wide bonds run one wave per SIMD regardless).
  Sched best;
  bool have = false;
  double best_score = 0.0;
  int first_ng = 0;
  const int occ_cap = h->chi >= 256 ? 1 : kPassOccupancy;
  for (int ng = 1; ng <= 64; ++ng) {
    if (first_ng && ng > first_ng + 3) break;
    for (int c = 0; c <= h->L; ++c) {
      Sched s = build_sched(h->pi, h->N, h->L, c, ng);
      const size_t lds = pass_lds_bytes(h->chi, s.nslot, h->nw, h->dtype);
      if (lds > kLdsLimit || s.nslot > pass_max_slots(h->dtype, h->chi)) continue;
      if (!first_ng) first_ng = ng;
      const int occ = std::min<int>(occ_cap, (int)(kLdsLimit / lds));
      const double score = (double)s.cost / occ;
      if (!have || score < best_score) { best = s; best_score = score; have = true; }
    }
  }
  if (!have) return fail(RTT_E_UNSUPPORTED, "rtt_create: flip-ratio rows of one walker exceed on-chip memory");
  if (chain_lds_bytes(h->chi, h->T, h->L, h->nw, h->N) > kLdsLimit)
    return fail(RTT_E_UNSUPPORTED, "rtt_create: sampling state of 16 walkers exceeds on-chip memory");
  h->sched = best;
  // proposal order: spins by first position, unread spins last
  h->first.assign(h->N, -1);
  for (int k = 0; k < h->L; ++k)
    if (h->first[h->pi[k]] < 0) h->first[h->pi[k]] = k;
  h->order.clear();
  for (int k = 0; k < h->L; ++k)
    if (h->first[h->pi[k]] == k) h->order.push_back(h->pi[k]);
  for (int j = 0; j < h->N; ++j)
    if (h->first[j] < 0) h->order.push_back(j);

  // pack and upload every term
  std::vector<uint8_t> fw_all, bw_all, fw, bw;
  for (int t = 0; t < h->T; ++t) {
    pack_term(h, t, h->qcores[t], fw, bw);
    fw_all.insert(fw_all.end(), fw.begin(), fw.end());
    bw_all.insert(bw_all.end(), bw.begin(), bw.end());
  }
  rtt_status st;
  if ((st = upload(&h->d_fwd, fw_all.data(), fw_all.size())) != RTT_OK) return st;
  if ((st = upload(&h->d_bwd, bw_all.data(), bw_all.size())) != RTT_OK) return st;
  if ((st = upload((void**)&h->d_cexp, h->core_exp.data(), h->core_exp.size() * 4)) != RTT_OK) return st;
  if ((st = upload((void**)&h->d_cesum, h->cesum.data(), h->cesum.size() * 4)) != RTT_OK) return st;
  if ((st = upload((void**)&h->d_rmask, h->rmask.data(), h->rmask.size() * 8)) != RTT_OK) return st;
  if ((st = upload((void**)&h->d_sf, best.fwd.data(), best.fwd.size() * 4)) != RTT_OK) return st;
  if ((st = upload((void**)&h->d_sb, best.bwd.data(), best.bwd.size() * 4)) != RTT_OK) return st;
  if ((st = upload((void**)&h->d_fslot, best.fslot.data(), best.fslot.size() * 4)) != RTT_OK) return st;
  if ((st = upload((void**)&h->d_bslot, best.bslot.data(), best.bslot.size() * 4)) != RTT_OK) return st;
  if ((st = upload((void**)&h->d_grp, best.grp.data(), best.grp.size() * 4)) != RTT_OK) return st;
  if ((st = upload((void**)&h->d_fgs, best.fgs.data(), best.fgs.size() * 4)) != RTT_OK) return st;
  if ((st = upload((void**)&h->d_bgs, best.bgs.data(), best.bgs.size() * 4)) != RTT_OK) return st;
  if ((st = upload((void**)&h->d_pi, h->pi.data(), h->pi.size() * 4)) != RTT_OK) return st;
  if ((st = upload((void**)&h->d_order, h->order.data(), h->order.size() * 4)) != RTT_OK) return st;
  if ((st = upload((void**)&h->d_first, h->first.data(), h->first.size() * 4)) != RTT_OK) return st;
  if ((st = upload((void**)&h->d_coeffs, h->coeffs.data(), h->coeffs.size() * 8)) != RTT_OK) return st;
  if ((st = setup_narrow(h)) != RTT_OK) return st;
  const char* ck = getenv("RTT_CHAIN_CHECKPOINTS");
  h->chain_ck = (ck && ck[0] == '0') ? 0 : 1;
  HIPX(hipDeviceSynchronize());
  return RTT_OK;
}

// Grow a workspace buffer in stream order (the stream-ordered allocator):
// the old buffer is released after the work already queued on `s`, the new
// one is ready for the work queued after it, and the device is never
// synchronised.  Workspace of a handle therefore belongs to one stream at a
// time.
rtt_status grow_async(void** p, size_t bytes, hipStream_t s) {
  if (*p) HIPX(hipFreeAsync(*p, s));
  *p = nullptr;
  HIPX(hipMallocAsync(p, std::max<size_t>(bytes, 16), s));
  return RTT_OK;
}

rtt_status ensure_ws(rtt_s* h, int W, hipStream_t s) {
  if ((size_t)W <= h->ws_W) return RTT_OK;
  h->ws_W = 0;
  const size_t rows = (size_t)h->T * h->sched.ng * W * h->sched.nslot;
  rtt_status st;
  if ((st = grow_async((void**)&h->d_u, rows * h->chi * 4, s)) != RTT_OK) return st;
  if ((st = grow_async((void**)&h->d_v, rows * h->chi * 4, s)) != RTT_OK) return st;
  if ((st = grow_async((void**)&h->d_ue, rows * 4, s)) != RTT_OK) return st;
  if ((st = grow_async((void**)&h->d_ve, rows * 4, s)) != RTT_OK) return st;
  h->ws_W = W;
  return RTT_OK;
}

// ------------------------------------------------------------------ dispatch
template <class D, int CHI>
rtt_status launch_pass(const rttk::PassArgs& a, int T, hipStream_t s) {
  constexpr int WPW = rttk::Geo<CHI>::WPW;
  constexpr int WPB = 4 / WPW;
  const size_t lds = pass_lds_bytes(CHI, a.nslot, a.nw,
                                    std::is_same<D, rttk::DFP8>::value    ? RTT_FP8_E4M3
                                    : std::is_same<D, rttk::DBF16>::value ? RTT_BF16
                                                                          : RTT_F32);
  auto kfn = rttk::pass_kernel<D, CHI>;
  HIPX(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  dim3 grid((a.W + WPB - 1) / WPB, T);
  hipLaunchKernelGGL(kfn, grid, dim3(256), lds, s, a);
  HIPX(hipGetLastError());
  return RTT_OK;
}

int device_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}

// Column checkpoints for a sweep launch: as many as fit in the LDS left over
// (without lowering the blocks per CU the launch needs, at most 16), evenly
// spaced over the bonds a proposal can start its columns from, [lo, L), lo
// being passed in ck_first.
void chain_checkpoints(rttk::ChainArgs& a, int chi, int cg, int blocks) {
  const int lo = a.ck_first, LW = (a.L + 63) / 64;
  a.n_ck = 0; a.ck_first = 0; a.ck_step = 1;
  if (a.mode != 1 || lo >= a.L || lo < 1) return;
  const rttk::ChainLayout l0(chi, a.T, LW, a.nw, cg, 0, a.N);
  int nmax = 0;
  if (l0.seq) {
    // sequential layout (bond 256, one block per CU): the vectors go to the
    // global buffer, only their exponents take LDS
    if (chi != 256 || cg != 1 || !a.ckg) return;
    for (int n = std::min(16, a.ck_cap); n >= 1 && nmax == 0; --n)
      if ((size_t)rttk::ChainLayout(chi, a.T, LW, a.nw, cg, n, a.N).total <= kLdsLimit) nmax = n;
  } else {
    if (chi > 64) return;
    const size_t budget = kLdsLimit / (blocks > device_cus() ? 2 : 1);
    // the largest count whose layout fits, preferring counts that keep the
    // replica bitmasks in LDS as they are without checkpoints (each layout is
    // sized in full: the masks may stop fitting as checkpoints are added)
    for (int pass = 0; pass < 2 && nmax == 0; ++pass)
      for (int n = 16; n >= 1; --n) {
        const rttk::ChainLayout ln(chi, a.T, LW, a.nw, cg, n, a.N);
        if ((size_t)ln.total <= budget && (pass == 1 || ln.rml == l0.rml)) { nmax = n; break; }
      }
  }
  if (nmax < 1) return;
  const int span = a.L - lo;
  const int step = (span + nmax - 1) / nmax;
  a.n_ck = (span + step - 1) / step;
  a.ck_first = lo;
  a.ck_step = step;
}

template <class D, int CHI, int CG>
rtt_status launch_chain_cg(const rttk::ChainArgs& a0, hipStream_t s) {
  rttk::ChainArgs a = a0;
  dim3 grid((a.W + 16 * CG - 1) / (16 * CG));
  chain_checkpoints(a, CHI, CG, (int)grid.x);
  const size_t lds = (size_t)rttk::ChainLayout(CHI, a.T, (a.L + 63) / 64, a.nw, CG, a.n_ck, a.N).total;
  auto kfn = rttk::chain_kernel<D, CHI, CG, false>;
  // (at bond 256 only the FP8 kernel fits the checkpoint code in registers;
  // the BF16 one would spill)
  if constexpr (CHI <= 64)
    if (a.n_ck > 0) kfn = rttk::chain_kernel<D, CHI, CG, true>;
  if constexpr (CHI == 256 && CG == 1 && std::is_same<D, rttk::DFP8>::value)
    if (a.n_ck > 0) kfn = rttk::chain_kernel<D, CHI, CG, true, true>;   // sequential layout: vectors in global memory
  HIPX(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(kfn, grid, dim3(rttk::ChainGeo<CHI, D>::NT), lds, s, a);
  HIPX(hipGetLastError());
  return RTT_OK;
}

// Bond 128 with enough walkers to give every CU a block of 32 runs two
// column groups per block (each core fragment serves 32 walkers), if the
// state still fits on chip in the same layout.  (At 256 the registers of a
// second group would spill; at 64 and below two waves share each SIMD.)
template <class D, int CHI>
rtt_status launch_chain(const rttk::ChainArgs& a, hipStream_t s) {
  if constexpr (CHI == 128) {
    const int LW = (a.L + 63) / 64;
    const rttk::ChainLayout l1(CHI, a.T, LW, a.nw, 1, 0, a.N), l2(CHI, a.T, LW, a.nw, 2, 0, a.N);
    if (a.W >= 32 * device_cus() && l2.seq == l1.seq && (size_t)l2.total <= kLdsLimit)
      return launch_chain_cg<D, CHI, 2>(a, s);
  }
  return launch_chain_cg<D, CHI, 1>(a, s);
}

template <template <class, int> class F, class... Args>
rtt_status dispatch(int dtype, int chi, Args&&... args) {
  if (dtype == RTT_F32) {
    switch (chi) {
      case 16: return F<rttk::DF32, 16>::run(args...);
      case 32: return F<rttk::DF32, 32>::run(args...);
      case 64: return F<rttk::DF32, 64>::run(args...);
      case 128: return F<rttk::DF32, 128>::run(args...);
    }
  } else if (dtype == RTT_BF16) {
    switch (chi) {
      case 32: return F<rttk::DBF16, 32>::run(args...);
      case 64: return F<rttk::DBF16, 64>::run(args...);
      case 128: return F<rttk::DBF16, 128>::run(args...);
      case 256: return F<rttk::DBF16, 256>::run(args...);
    }
  } else if (dtype == RTT_FP8_E4M3) {
    switch (chi) {
      case 32: return F<rttk::DFP8, 32>::run(args...);
      case 64: return F<rttk::DFP8, 64>::run(args...);
      case 128: return F<rttk::DFP8, 128>::run(args...);
      case 256: return F<rttk::DFP8, 256>::run(args...);
    }
  }
  return fail(RTT_E_UNSUPPORTED, "no kernel for dtype %d, padded bond %d", dtype, chi);
}

template <class D, int CHI>
struct PassL {
  static rtt_status run(const rttk::PassArgs& a, int T, hipStream_t s) { return launch_pass<D, CHI>(a, T, s); }
};
template <class D, int CHI>
struct ChainL {
  static rtt_status run(const rttk::ChainArgs& a, hipStream_t s) { return launch_chain<D, CHI>(a, s); }
};

// nearest-neighbour bonds (i, i + x) and (i, i + y); wrap bonds on sides >= 3
std::vector<int2> tfim_bond_list(int Lx, int Ly, int periodic) {
  std::vector<int2> b;
  for (int y = 0; y < Ly; ++y)
    for (int x = 0; x < Lx; ++x) {
      const int i = y * Lx + x;
      if (x + 1 < Lx) b.push_back(make_int2(i, y * Lx + x + 1));
      else if (periodic && Lx >= 3) b.push_back(make_int2(i, y * Lx));
      if (y + 1 < Ly) b.push_back(make_int2(i, (y + 1) * Lx + x));
      else if (periodic && Ly >= 3) b.push_back(make_int2(i, x));
    }
  return b;
}

// read a host train (rtt_create layout) with its bonds checked
rtt_status read_train(const char* who, int32_t L, const int32_t* bond, const double* cores, rtt_tt::Train& t) {
  if (L < 1 || !bond || !cores) return fail(RTT_E_ARG, "%s: empty train or null pointer", who);
  if (bond[0] != 1 || bond[L] != 1) return fail(RTT_E_ARG, "%s: boundary bonds must be 1", who);
  t.bond.assign(bond, bond + L + 1);
  t.core.resize(L);
  size_t off = 0;
  for (int k = 0; k < L; ++k) {
    if (bond[k] < 1 || bond[k] > 4096) return fail(RTT_E_ARG, "%s: bond[%d] = %d", who, k, bond[k]);
    const size_t n = (size_t)2 * bond[k] * bond[k + 1];
    t.core[k].assign(cores + off, cores + off + n);
    for (double x : t.core[k])
      if (!isfinite(x)) return fail(RTT_E_ARG, "%s: non-finite core entry at position %d", who, k);
    off += n;
  }
  return RTT_OK;
}

rtt_status write_train(const char* who, const rtt_tt::Train& t, int32_t* bond_out, double* cores_out, int64_t cap,
                       int64_t* n_out) {
  int64_t need = 0;
  for (int k = 0; k < t.L(); ++k) need += (int64_t)t.core[k].size();
  if (n_out) *n_out = need;
  if (!bond_out || !cores_out || cap < need)
    return fail(RTT_E_ARG, "%s: output needs %lld doubles, capacity %lld", who, (long long)need, (long long)cap);
  for (int k = 0; k <= t.L(); ++k) bond_out[k] = t.bond[k];
  int64_t off = 0;
  for (int k = 0; k < t.L(); ++k) {
    std::copy(t.core[k].begin(), t.core[k].end(), cores_out + off);
    off += (int64_t)t.core[k].size();
  }
  return RTT_OK;
}

rtt_status check_handle(const rtt_s* h) {
  if (!h) return fail(RTT_E_ARG, "null RTT handle");
  return RTT_OK;
}

rttn::NarrowArgs narrow_args(const rtt_s* h, int W) {
  rttn::NarrowArgs a{};
  a.cores = h->d_ncores; a.cesum = h->d_cesum; a.rmask = h->d_rmask; a.pi = h->d_pi;
  a.order = h->d_order; a.first = h->d_first; a.coeffs = h->d_coeffs;
  a.T = h->T; a.L = h->L; a.N = h->N; a.nw = h->nw; a.LW = (h->L + 63) / 64; a.W = W;
  return a;
}

template <int C>
rtt_status launch_narrow_eval(const rttn::NarrowArgs& a, hipStream_t s) {
  const int threads = std::min(1024, (a.N + 1 + 63) / 64 * 64);
  hipLaunchKernelGGL(rttn::narrow_eval_kernel<C>, dim3(a.W), dim3(threads), (size_t)a.LW * 8, s, a);
  HIPX(hipGetLastError());
  return RTT_OK;
}

// Segmented sampling (one term, L <= 4096): G lanes per walker, segments
// of at most 64 positions.  More lanes shorten the chain of dependent
// products per proposal but add tree levels and lanes; G is chosen so that
// the launch holds about two waves per SIMD (8 per CU), which measured best
// on the 400-position chi = 2 train at 4096 walkers (G = 32) and at 16384
// (G = 8).
size_t narrow_seg_lds(const rtt_s* h, int G) {
  return ((size_t)h->L * 2 * h->narrow * h->narrow * 4 + 7) / 8 * 8 + (size_t)(64 / G) * h->nw * 8;
}

int narrow_seg_lanes(const rtt_s* h, int W) {
  if (h->T != 1 || h->L > 64 * 64) return 0;
  int gmin = 1;
  while (gmin * 64 < h->L) gmin <<= 1;
  const long lanes = (long)device_cus() * 8 * 64;
  int G = 1;
  while (G < 64 && (long)W * G * 2 <= lanes) G <<= 1;
  G = std::max(G, gmin);
  return narrow_seg_lds(h, G) <= kLdsLimit ? G : 0;
}

template <int C, int G>
rtt_status launch_seg(const rttn::NarrowArgs& a, size_t lds, hipStream_t s) {
  auto kfn = rttn::narrow_chain_seg_kernel<C, G>;
  HIPX(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  constexpr int WPB = 64 / G;
  hipLaunchKernelGGL(kfn, dim3((a.W + WPB - 1) / WPB), dim3(64), lds, s, a);
  HIPX(hipGetLastError());
  return RTT_OK;
}

template <int C>
rtt_status launch_seg_g(const rttn::NarrowArgs& a, int G, size_t lds, hipStream_t s) {
  switch (G) {
    case 1: return launch_seg<C, 1>(a, lds, s);
    case 2: return launch_seg<C, 2>(a, lds, s);
    case 4: return launch_seg<C, 4>(a, lds, s);
    case 8: return launch_seg<C, 8>(a, lds, s);
    case 16: return launch_seg<C, 16>(a, lds, s);
    case 32: return launch_seg<C, 32>(a, lds, s);
    case 64: return launch_seg<C, 64>(a, lds, s);
  }
  return fail(RTT_E_UNSUPPORTED, "segmented sampling: %d lanes per walker", G);
}

template <int C>
rtt_status launch_narrow_chain(const rttn::NarrowArgs& a, size_t lds, hipStream_t s) {
  auto kfn = rttn::narrow_chain_kernel<C>;
  HIPX(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(kfn, dim3((a.W + 63) / 64), dim3(64), lds, s, a);
  HIPX(hipGetLastError());
  return RTT_OK;
}

// The host tensor-train algebra allocates freely: a failed allocation, or
// any other exception, becomes a status code instead of crossing the C ABI.
template <class F>
rtt_status host_guard(const char* who, F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(RTT_E_OOM, "%s: host memory exhausted", who);
  } catch (const std::exception& e) {
    return fail(RTT_E_ARG, "%s: %s", who, e.what());
  }
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* rtt_last_error(void) { return g_err.c_str(); }

int32_t rtt_abi_version(void) { return 3; }

static rtt_status rtt_create_impl(int32_t n_spins, int32_t n_cores, const int32_t* pi, const int32_t* bond,
                      const double* cores, int32_t dtype, rtt_t* out) {
  g_err.clear();
  if (!out) return fail(RTT_E_ARG, "rtt_create: out is null");
  *out = nullptr;
  if (n_spins < 1 || n_spins > 1024) return fail(RTT_E_ARG, "rtt_create: n_spins %d outside [1, 1024]", n_spins);
  if (n_cores < 1) return fail(RTT_E_ARG, "rtt_create: n_cores %d < 1", n_cores);
  if (!pi || !bond || !cores) return fail(RTT_E_ARG, "rtt_create: null pointer argument");
  if (dtype != RTT_F32 && dtype != RTT_BF16 && dtype != RTT_FP8_E4M3)
    return fail(RTT_E_ARG, "rtt_create: unknown dtype %d", dtype);
  for (int k = 0; k < n_cores; ++k)
    if (pi[k] < 0 || pi[k] >= n_spins) return fail(RTT_E_ARG, "rtt_create: pi[%d] = %d outside [0, %d)", k, pi[k], n_spins);
  if (bond[0] != 1 || bond[n_cores] != 1) return fail(RTT_E_ARG, "rtt_create: boundary bonds must be 1");
  int bmax = 1;
  for (int k = 0; k <= n_cores; ++k) {
    if (bond[k] < 1 || bond[k] > 256) return fail(RTT_E_ARG, "rtt_create: bond[%d] = %d outside [1, 256]", k, bond[k]);
    bmax = std::max(bmax, (int)bond[k]);
  }
  const int chi = std::max(dtype == RTT_F32 ? 16 : 32, next_pow2(bmax));
  if (dtype == RTT_F32 && chi > 128) return fail(RTT_E_UNSUPPORTED, "rtt_create: FP32 supports bonds up to 128");
  size_t ncore = 0;
  for (int k = 0; k < n_cores; ++k) ncore += (size_t)2 * bond[k] * bond[k + 1];
  for (size_t i = 0; i < ncore; ++i)
    if (!isfinite(cores[i])) return fail(RTT_E_ARG, "rtt_create: non-finite core entry %zu", i);

  rtt_s* h = new rtt_s;
  h->N = n_spins;
  h->L = n_cores;
  h->chi = chi;
  h->dtype = dtype;
  h->T = 1;
  h->nw = (n_spins + 63) / 64;
  h->pi.assign(pi, pi + n_cores);
  h->bond.assign(bond, bond + n_cores + 1);
  h->coeffs = {1.0};
  h->qcores.resize(1);
  h->fp8e.resize(1);
  quantise(dtype, h->bond, cores, h->qcores[0], h->fp8e[0]);
  (void)hipGetDevice(&h->device);
  rtt_status st = finish_create(h);
  if (st != RTT_OK) {
    free_dev(h);
    delete h;
    return st;
  }
  *out = h;
  return RTT_OK;
}

static rtt_status rtt_lincomb_impl(int32_t n_terms, const rtt_t* terms, const double* coeffs, rtt_t* out) {
  g_err.clear();
  if (!out) return fail(RTT_E_ARG, "rtt_lincomb: out is null");
  *out = nullptr;
  if (n_terms < 1 || n_terms > rttk::kMaxTerms) return fail(RTT_E_ARG, "rtt_lincomb: n_terms %d outside [1, %d]", n_terms, rttk::kMaxTerms);
  if (!terms || !coeffs) return fail(RTT_E_ARG, "rtt_lincomb: null pointer argument");
  const rtt_s* t0 = terms[0];
  if (!t0) return fail(RTT_E_ARG, "rtt_lincomb: null term 0");
  for (int t = 0; t < n_terms; ++t) {
    const rtt_s* x = terms[t];
    if (!x) return fail(RTT_E_ARG, "rtt_lincomb: null term %d", t);
    if (x->T != 1) return fail(RTT_E_ARG, "rtt_lincomb: term %d is itself a combination", t);
    if (x->N != t0->N || x->L != t0->L || x->pi != t0->pi || x->chi != t0->chi || x->dtype != t0->dtype)
      return fail(RTT_E_ARG, "rtt_lincomb: term %d differs from term 0 in N, L, pi, bond or dtype", t);
    if (!isfinite(coeffs[t])) return fail(RTT_E_ARG, "rtt_lincomb: coefficient %d not finite", t);
  }
  rtt_s* h = new rtt_s;
  h->N = t0->N;
  h->L = t0->L;
  h->chi = t0->chi;
  h->dtype = t0->dtype;
  h->T = n_terms;
  h->nw = t0->nw;
  h->pi = t0->pi;
  h->bond = t0->bond;
  // terms may have different inner bonds: keep each term's own layout
  h->coeffs.assign(coeffs, coeffs + n_terms);
  for (int t = 0; t < n_terms; ++t) {
    h->qcores.push_back(terms[t]->qcores[0]);
    h->fp8e.push_back(terms[t]->fp8e[0]);
  }
  // pack_term reads bond per handle: all terms share bond only if equal; pad via each term
  bool same_bond = true;
  for (int t = 0; t < n_terms; ++t) same_bond &= (terms[t]->bond == t0->bond);
  if (!same_bond) {
    delete h;
    return fail(RTT_E_ARG, "rtt_lincomb: terms must share the bond dimensions");
  }
  (void)hipGetDevice(&h->device);
  rtt_status st = finish_create(h);
  if (st != RTT_OK) {
    free_dev(h);
    delete h;
    return st;
  }
  *out = h;
  return RTT_OK;
}

rtt_status rtt_destroy(rtt_t h) {
  g_err.clear();
  if (!h) return RTT_OK;
  HIPX(hipDeviceSynchronize());
  free_dev(h);
  delete h;
  return RTT_OK;
}

rtt_status rtt_info(rtt_t h, int32_t* info) {
  if (check_handle(h) != RTT_OK) return RTT_E_ARG;
  if (!info) return fail(RTT_E_ARG, "rtt_info: info is null");
  info[0] = h->N; info[1] = h->L; info[2] = h->chi; info[3] = h->dtype;
  info[4] = h->T; info[5] = h->nw; info[6] = h->sched.cut; info[7] = h->sched.nslot;
  info[8] = h->sched.ng; info[9] = h->narrow;
  return RTT_OK;
}

// Quantised core values of one term as the device uses them (host double,
// rtt_create layout, FP8 scale applied).  Read back from device memory and
// unpacked, so it also checks the fragment packing.
rtt_status rtt_get_cores(rtt_t h, int32_t term, double* out) {
  if (check_handle(h) != RTT_OK) return RTT_E_ARG;
  if (!out || term < 0 || term >= h->T) return fail(RTT_E_ARG, "rtt_get_cores: bad argument");
  const int chi = h->chi, L = h->L, KPL = chi / 4;
  const size_t eb = elem_bytes(h->dtype), slice = (size_t)chi * chi;
  std::vector<uint8_t> fw((size_t)L * 2 * slice * eb);
  HIPX(hipMemcpy(fw.data(), (const uint8_t*)h->d_fwd + (size_t)term * fw.size(), fw.size(), hipMemcpyDeviceToHost));
  size_t off = 0;
  for (int k = 0; k < L; ++k) {
    const int a = h->bond[k], b = h->bond[k + 1];
    const double scale = ldexp(1.0, h->core_exp[(size_t)term * L + k]);
    for (int s = 0; s < 2; ++s)
      for (int i = 0; i < a; ++i)
        for (int j = 0; j < b; ++j) {
          // forward layout holds core[s][i][j] at g*KPL+e = i, 16t+m = j
          const int g = i / KPL, e = i % KPL, t = j / 16, m = j % 16;
          const size_t idx = ((size_t)k * 2 + s) * slice + (size_t)t * 64 * KPL +
                             rttk::frag_offset(16 * g + m, e, rttk::frag_chunk((int)eb, KPL));
          double v;
          if (eb == 4) { float f; memcpy(&f, &fw[idx * 4], 4); v = f; }
          else if (eb == 1) v = e4m3_decode(fw[idx]) / 512.0;
          else { uint16_t u; memcpy(&u, &fw[idx * 2], 2); v = bf16_value(u); }
          out[off + ((size_t)s * a + i) * b + j] = v * scale;
        }
    off += (size_t)2 * a * b;
  }
  return RTT_OK;
}

static rtt_status rtt_tfim_create_impl(int32_t Lx, int32_t Ly, int32_t periodic, double J, double h, rtt_ham_t* out) {
  g_err.clear();
  if (!out) return fail(RTT_E_ARG, "rtt_tfim_create: out is null");
  *out = nullptr;
  if (Lx < 1 || Ly < 1 || (long)Lx * Ly > 1024) return fail(RTT_E_ARG, "rtt_tfim_create: bad lattice %dx%d", Lx, Ly);
  if (!isfinite(J) || !isfinite(h)) return fail(RTT_E_ARG, "rtt_tfim_create: J and h must be finite");
  const std::vector<int2> b = tfim_bond_list(Lx, Ly, periodic);
  rtt_ham_s* H = new rtt_ham_s;
  H->Lx = Lx; H->Ly = Ly; H->periodic = periodic; H->J = J; H->h = h; H->nb = (int)b.size();
  rtt_status st = upload((void**)&H->d_bonds, b.data(), b.size() * sizeof(int2));
  if (st != RTT_OK) { delete H; return st; }
  *out = H;
  return RTT_OK;
}

rtt_status rtt_tfim_destroy(rtt_ham_t H) {
  if (!H) return RTT_OK;
  HIPX(hipDeviceSynchronize());
  if (H->d_bonds) (void)hipFree(H->d_bonds);
  delete H;
  return RTT_OK;
}

}  // extern "C"

namespace {

// Workspace of the flip-ratio passes: forward and backward cut vectors and
// their exponents, [T][groups][W][slots] each.
struct EvalWs {
  float* u; float* v; int* ue; int* ve;
};

size_t eval_ws_rows(const rtt_s* h, int W) { return (size_t)h->T * h->sched.ng * W * h->sched.nslot; }
size_t eval_ws_bytes(const rtt_s* h, int W) { return eval_ws_rows(h, W) * 2 * ((size_t)h->chi * 4 + 4); }

rtt_status check_eval_args(const char* who, rtt_t h, rtt_ham_t ham, int32_t W, const uint64_t* spins,
                           const double* eloc) {
  if (check_handle(h) != RTT_OK) return RTT_E_ARG;
  if (W < 1) return fail(RTT_E_ARG, "%s: W = %d < 1", who, W);
  if (!spins) return fail(RTT_E_ARG, "%s: spins is null", who);
  if (eloc && !ham) return fail(RTT_E_ARG, "%s: eloc requested without a Hamiltonian", who);
  if (ham && ham->Lx * ham->Ly != h->N)
    return fail(RTT_E_ARG, "%s: lattice has %d sites, RTT has %d spins", who, ham->Lx * ham->Ly, h->N);
  return RTT_OK;
}

// The evaluation itself on a given workspace (unused by narrow-bond trains).
rtt_status evaluate_on(rtt_t h, rtt_ham_t ham, int32_t W, const uint64_t* spins, double* logabs, int8_t* sign,
                       double* logratio, int8_t* rsign, double* eloc, int32_t* status, const EvalWs& ws,
                       hipStream_t s) {
  if (h->narrow) {
    rttn::NarrowArgs na = narrow_args(h, W);
    na.spins = const_cast<uint64_t*>(spins);
    na.bonds = ham ? ham->d_bonds : nullptr;
    na.nbonds = ham ? ham->nb : 0;
    na.J = ham ? ham->J : 0.0;
    na.h = ham ? ham->h : 0.0;
    na.logabs = logabs; na.sign = sign; na.logratio = logratio; na.rsign = rsign; na.eloc = eloc;
    na.status = status;
    return h->narrow == 2 ? launch_narrow_eval<2>(na, s) : launch_narrow_eval<4>(na, s);
  }
  rtt_status st;
  rttk::PassArgs pa{};
  pa.core_exp = h->d_cexp;
  pa.nslot = h->sched.nslot;
  pa.L = h->L;
  pa.nw = h->nw;
  pa.W = W;
  pa.spins = spins;
  // forward
  pa.ng = h->sched.ng;
  pa.cores = h->d_fwd;
  pa.sched = h->d_sf;
  pa.gsteps = h->d_fgs;
  pa.out_vec = ws.u;
  pa.out_exp = ws.ue;
  if ((st = dispatch<PassL>(h->dtype, h->chi, pa, h->T * h->sched.ng, s)) != RTT_OK) return st;
  // backward
  pa.cores = h->d_bwd;
  pa.sched = h->d_sb;
  pa.gsteps = h->d_bgs;
  pa.out_vec = ws.v;
  pa.out_exp = ws.ve;
  if ((st = dispatch<PassL>(h->dtype, h->chi, pa, h->T * h->sched.ng, s)) != RTT_OK) return st;
  rttk::CombineArgs ca{};
  ca.u = ws.u; ca.ue = ws.ue; ca.v = ws.v; ca.ve = ws.ve;
  ca.nsf = h->sched.nslot; ca.nsb = h->sched.nslot; ca.chi = h->chi; ca.T = h->T; ca.W = W;
  ca.N = h->N; ca.nw = h->nw; ca.fslot = h->d_fslot; ca.bslot = h->d_bslot; ca.coeffs = h->d_coeffs;
  ca.ng = h->sched.ng; ca.grp = h->d_grp;
  ca.spins = spins;
  ca.bonds = ham ? ham->d_bonds : nullptr;
  ca.nbonds = ham ? ham->nb : 0;
  ca.J = ham ? ham->J : 0.0;
  ca.h = ham ? ham->h : 0.0;
  ca.logabs = logabs; ca.sign = sign; ca.logratio = logratio; ca.rsign = rsign; ca.eloc = eloc; ca.status = status;
  hipLaunchKernelGGL(rttk::combine_kernel, dim3((W + 3) / 4), dim3(256), 0, s, ca);
  HIPX(hipGetLastError());
  return RTT_OK;
}

// Workspace of rtt_evaluate_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  In host code `scratch` only names the
// symbol; its device address comes from hipGetSymbolAddress, once per
// device, with that device current.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

rtt_status scratch_address(void** out) {
  int dev = 0;
  HIPX(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(RTT_E_UNSUPPORTED, "device %d: more devices than the library keeps", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPX(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(RTT_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RTT_OK;
}

}  // namespace

extern "C" {

rtt_status rtt_evaluate(rtt_t h, rtt_ham_t ham, int32_t W, const uint64_t* spins, double* logabs,
                        int8_t* sign, double* logratio, int8_t* rsign, double* eloc, int32_t* status,
                        void* stream) {
  g_err.clear();
  rtt_status st = check_eval_args("rtt_evaluate", h, ham, W, spins, eloc);
  if (st != RTT_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (!h->narrow && (st = ensure_ws(h, W, s)) != RTT_OK) return st;
  return evaluate_on(h, ham, W, spins, logabs, sign, logratio, rsign, eloc, status,
                     EvalWs{h->d_u, h->d_v, h->d_ue, h->d_ve}, s);
}

rtt_status rtt_evaluate_noalloc(rtt_t h, rtt_ham_t ham, int32_t W, const uint64_t* spins, double* logabs,
                                int8_t* sign, double* logratio, int8_t* rsign, double* eloc,
                                int32_t* status, void* stream) {
  g_err.clear();
  rtt_status st = check_eval_args("rtt_evaluate_noalloc", h, ham, W, spins, eloc);
  if (st != RTT_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  EvalWs ws{nullptr, nullptr, nullptr, nullptr};
  if (!h->narrow) {
    const size_t need = eval_ws_bytes(h, W);
    if (need > kScratchBytes) {
      const size_t per = eval_ws_bytes(h, 1);
      return fail(RTT_E_ARG, "rtt_evaluate_noalloc: %d walkers need %zu bytes of workspace, more than the %zu "
                  "bytes held for it (at most %zu walkers of this state per call)", W, need, kScratchBytes,
                  kScratchBytes / per);
    }
    void* base = nullptr;
    if ((st = scratch_address(&base)) != RTT_OK) return st;
    const size_t rows = eval_ws_rows(h, W), vec = rows * h->chi * 4;
    unsigned char* b = static_cast<unsigned char*>(base);
    ws.u = reinterpret_cast<float*>(b);
    ws.v = reinterpret_cast<float*>(b + vec);
    ws.ue = reinterpret_cast<int*>(b + 2 * vec);
    ws.ve = reinterpret_cast<int*>(b + 2 * vec + rows * 4);
  }
  return evaluate_on(h, ham, W, spins, logabs, sign, logratio, rsign, eloc, status, ws, s);
}

rtt_status rtt_flip_ratios(rtt_t h, int32_t W, const uint64_t* spins, double* logratio, int8_t* rsign,
                           void* stream) {
  return rtt_evaluate(h, nullptr, W, spins, nullptr, nullptr, logratio, rsign, nullptr, nullptr, stream);
}

rtt_status rtt_local_energy(rtt_t h, rtt_ham_t ham, int32_t W, const uint64_t* spins, double* eloc,
                            void* stream) {
  if (!eloc) return fail(RTT_E_ARG, "rtt_local_energy: eloc is null");
  return rtt_evaluate(h, ham, W, spins, nullptr, nullptr, nullptr, nullptr, eloc, nullptr, stream);
}

static rtt_status chain_common(rtt_t h, int32_t W, uint64_t* spins, double* logabs, int8_t* sign,
                               uint64_t seed, uint64_t rstream, uint64_t sweep0, int32_t n_sweeps,
                               uint32_t* accepts, int32_t* status, int mode, void* stream) {
  if (check_handle(h) != RTT_OK) return RTT_E_ARG;
  if (W < 1) return fail(RTT_E_ARG, "W = %d < 1", W);
  if (!spins) return fail(RTT_E_ARG, "spins is null");
  if (n_sweeps < 0) return fail(RTT_E_ARG, "n_sweeps = %d < 0", n_sweeps);
  if (h->narrow) {
    rttn::NarrowArgs na = narrow_args(h, W);
    na.spins = spins; na.logabs = logabs; na.sign = sign; na.accepts = accepts; na.status = status;
    na.seed = seed; na.rstream = rstream; na.sweep0 = sweep0; na.n_sweeps = n_sweeps; na.mode = mode;
    const int G = narrow_seg_lanes(h, W);
    if (G) {
      const size_t lds = narrow_seg_lds(h, G);
      return h->narrow == 2 ? launch_seg_g<2>(na, G, lds, (hipStream_t)stream)
                            : launch_seg_g<4>(na, G, lds, (hipStream_t)stream);
    }
    const size_t lds = narrow_chain_lds(h);
    return h->narrow == 2 ? launch_narrow_chain<2>(na, lds, (hipStream_t)stream)
                          : launch_narrow_chain<4>(na, lds, (hipStream_t)stream);
  }
  rttk::ChainArgs ca{};
  ca.cores = h->d_fwd; ca.cores_bwd = h->d_bwd;
  ca.cesum = h->d_cesum;
  ca.rmask = h->d_rmask;
  ca.pi = h->d_pi; ca.order = h->d_order; ca.first = h->d_first; ca.coeffs = h->d_coeffs;
  ca.T = h->T; ca.L = h->L; ca.N = h->N; ca.nw = h->nw; ca.LW = (h->L + 63) / 64; ca.W = W;
  ca.spins = spins; ca.logabs = logabs; ca.sign = sign; ca.accepts = accepts; ca.status = status;
  ca.seed = seed; ca.rstream = rstream; ca.sweep0 = sweep0; ca.n_sweeps = n_sweeps; ca.mode = mode;
  // Sequential sampler layout at bond 256 with FP8 cores (the terms of a
  // combination take turns): room for 8 column checkpoints per block in
  // global memory, grown
  // in stream order (8 checkpoints keep 0.72 of the dependent steps of
  // contracting every proposal's columns from the right boundary on the
  // 16x16 two-replica path; 16 would keep 0.70 at twice the memory)
  ca.ckg = nullptr;
  ca.ck_cap = 0;
  if (mode == 1 && h->chain_ck && h->chi == 256 && h->dtype == RTT_FP8_E4M3 &&
      rttk::ChainLayout(h->chi, h->T, (h->L + 63) / 64, h->nw, 1, 0, h->N).seq) {
    const int cap = 8;
    const size_t need = (size_t)((W + 15) / 16) * 2 * cap * h->T * 16 * (h->chi + 4) * 4;
    if (need > h->ck_bytes) {
      h->ck_bytes = 0;
      rtt_status st = grow_async((void**)&h->d_ck, need, (hipStream_t)stream);
      if (st != RTT_OK) return st;
      h->ck_bytes = need;
    }
    ca.ckg = h->d_ck;
    ca.ck_cap = cap;
  }
  // the lowest bond a proposal's columns can start from: one past the
  // smallest last position over the spins
  {
    std::vector<int> last(h->N, -1);
    for (int k = 0; k < h->L; ++k) last[h->pi[k]] = k;
    int lo = h->L;
    for (int j = 0; j < h->N; ++j)
      if (last[j] >= 0) lo = std::min(lo, last[j] + 1);
    ca.ck_first = h->chain_ck ? lo : h->L;
  }
  return dispatch<ChainL>(h->dtype, h->chi, ca, (hipStream_t)stream);
}

rtt_status rtt_amplitudes(rtt_t h, int32_t W, const uint64_t* spins, double* logabs, int8_t* sign,
                          void* stream) {
  g_err.clear();
  return chain_common(h, W, const_cast<uint64_t*>(spins), logabs, sign, 0, 0, 0, 0, nullptr, nullptr, 0,
                      stream);
}

rtt_status rtt_mcmc_sweep(rtt_t h, int32_t W, uint64_t* spins, double* logabs, int8_t* sign, uint64_t seed,
                          uint64_t rng_stream, uint64_t sweep0, int32_t n_sweeps, uint32_t* accepts,
                          int32_t* status, void* stream) {
  g_err.clear();
  return chain_common(h, W, spins, logabs, sign, seed, rng_stream, sweep0, n_sweeps, accepts, status, 1,
                      stream);
}

rtt_status rtt_mixed_estimators(int32_t M, const rtt_t* targets, rtt_ham_t ham, int32_t W,
                                const uint64_t* spins, const double* logabs_a, const int8_t* sign_a,
                                double* ratio, double* mixed, int32_t* status, void* stream) {
  g_err.clear();
  if (M < 1 || !targets) return fail(RTT_E_ARG, "rtt_mixed_estimators: M = %d targets", M);
  if (!ham) return fail(RTT_E_ARG, "rtt_mixed_estimators: Hamiltonian is null");
  if (W < 1) return fail(RTT_E_ARG, "rtt_mixed_estimators: W = %d < 1", W);
  if (!spins || !logabs_a || !sign_a || !ratio || !mixed)
    return fail(RTT_E_ARG, "rtt_mixed_estimators: null device pointer");
  for (int m = 0; m < M; ++m) {
    if (check_handle(targets[m]) != RTT_OK) return RTT_E_ARG;
    if (targets[m]->N != ham->Lx * ham->Ly)
      return fail(RTT_E_ARG, "rtt_mixed_estimators: target %d has %d spins, lattice %d sites", m,
                  targets[m]->N, ham->Lx * ham->Ly);
    if (targets[m]->N != targets[0]->N)
      return fail(RTT_E_ARG, "rtt_mixed_estimators: targets differ in spin count");
  }
  hipStream_t s = (hipStream_t)stream;
  for (int m = 0; m < M; ++m) {
    rtt_s* b = targets[m];
    if ((size_t)W > b->mix_W) {
      b->mix_W = 0;
      rtt_status st;
      if ((st = grow_async((void**)&b->d_mla, (size_t)W * 8, s)) != RTT_OK) return st;
      if ((st = grow_async((void**)&b->d_msg, (size_t)W, s)) != RTT_OK) return st;
      if ((st = grow_async((void**)&b->d_mel, (size_t)W * 8, s)) != RTT_OK) return st;
      if ((st = grow_async((void**)&b->d_mst, (size_t)W * 4, s)) != RTT_OK) return st;
      b->mix_W = W;
    }
    rtt_status st = rtt_evaluate(b, ham, W, spins, b->d_mla, b->d_msg, nullptr, nullptr, b->d_mel, b->d_mst,
                                 stream);
    if (st != RTT_OK) return st;
    hipLaunchKernelGGL(rttk::mixed_kernel, dim3((W + 255) / 256), dim3(256), 0, s, W, logabs_a, sign_a,
                       b->d_mla, b->d_msg, b->d_mel, b->d_mst, ratio + (size_t)m * W, mixed + (size_t)m * W,
                       status, m == 0 ? 1 : 0);
    HIPX(hipGetLastError());
  }
  return RTT_OK;
}

static rtt_status rtt_tt_round_impl(int32_t n_cores, const int32_t* bond, const double* cores, int32_t chi_max,
                        double rel_tol, int32_t* bond_out, double* cores_out, int64_t cap, int64_t* n_out) {
  g_err.clear();
  if (chi_max < 1 || !(rel_tol >= 0.0)) return fail(RTT_E_ARG, "rtt_tt_round: chi_max %d, rel_tol %g", chi_max, rel_tol);
  rtt_tt::Train t;
  rtt_status st = read_train("rtt_tt_round", n_cores, bond, cores, t);
  if (st != RTT_OK) return st;
  rtt_tt::round_train(t, chi_max, rel_tol);
  return write_train("rtt_tt_round", t, bond_out, cores_out, cap, n_out);
}

static rtt_status rtt_tfim_power_step_impl(int32_t n_spins, int32_t n_cores, const int32_t* pi, const int32_t* bond,
                               const double* cores, int32_t Lx, int32_t Ly, int32_t periodic, double J, double h,
                               double tau, int32_t chi_max, double rel_tol, int32_t* bond_out, double* cores_out,
                               int64_t cap, int64_t* n_out) {
  g_err.clear();
  if (Lx < 1 || Ly < 1 || Lx * Ly != n_spins)
    return fail(RTT_E_ARG, "rtt_tfim_power_step: lattice %dx%d for %d spins", Lx, Ly, n_spins);
  if (!isfinite(J) || !isfinite(h) || !isfinite(tau)) return fail(RTT_E_ARG, "rtt_tfim_power_step: non-finite J, h or tau");
  if (chi_max < 1 || !(rel_tol >= 0.0)) return fail(RTT_E_ARG, "rtt_tfim_power_step: chi_max %d, rel_tol %g", chi_max, rel_tol);
  if (!pi) return fail(RTT_E_ARG, "rtt_tfim_power_step: pi is null");
  std::vector<int> p(pi, pi + std::max(n_cores, 0));
  std::vector<int> seen(std::max(n_spins, 0), 0);
  for (int k = 0; k < n_cores; ++k) {
    if (p[k] < 0 || p[k] >= n_spins) return fail(RTT_E_ARG, "rtt_tfim_power_step: pi[%d] = %d", k, p[k]);
    seen[p[k]] = 1;
  }
  for (int j = 0; j < n_spins; ++j)
    if (!seen[j]) return fail(RTT_E_ARG, "rtt_tfim_power_step: spin %d is read by no position", j);
  rtt_tt::Train t;
  rtt_status st = read_train("rtt_tfim_power_step", n_cores, bond, cores, t);
  if (st != RTT_OK) return st;
  std::vector<std::pair<int, int>> bonds;
  for (const int2& b : tfim_bond_list(Lx, Ly, periodic)) bonds.push_back({b.x, b.y});
  const rtt_tt::Train out = rtt_tt::tfim_power_step(t, p, n_spins, bonds, J, h, tau, chi_max, rel_tol);
  return write_train("rtt_tfim_power_step", out, bond_out, cores_out, cap, n_out);
}

static rtt_status rtt_pauli_apply_impl(int32_t n_cores, const int32_t* bond, const double* cores, int32_t n_terms,
                           const double* coeffs, const uint8_t* ops, double alpha, double beta, int32_t chi_max,
                           int32_t chi_sum, double rel_tol, int32_t* bond_out, double* cores_out, int64_t cap, int64_t* n_out) {
  g_err.clear();
  if (n_terms < 1 || !coeffs || !ops) return fail(RTT_E_ARG, "rtt_pauli_apply: no terms or null pointer");
  if (!isfinite(alpha) || !isfinite(beta)) return fail(RTT_E_ARG, "rtt_pauli_apply: non-finite alpha or beta");
  if (chi_max < 1 || chi_sum < 1 || !(rel_tol >= 0.0))
    return fail(RTT_E_ARG, "rtt_pauli_apply: chi_max %d, chi_sum %d, rel_tol %g", chi_max, chi_sum, rel_tol);
  for (int t = 0; t < n_terms; ++t)
    if (!isfinite(coeffs[t])) return fail(RTT_E_ARG, "rtt_pauli_apply: coeffs[%d] is not finite", t);
  rtt_tt::Train t;
  rtt_status st = read_train("rtt_pauli_apply", n_cores, bond, cores, t);
  if (st != RTT_OK) return st;
  for (int64_t e = 0; e < (int64_t)n_terms * n_cores; ++e)
    if (ops[e] > 3)
      return fail(RTT_E_ARG, "rtt_pauli_apply: ops[%lld][%lld] = %d (0..3)", (long long)(e / n_cores),
                  (long long)(e % n_cores), ops[e]);
  const rtt_tt::Train out = rtt_tt::pauli_apply(t, n_terms, coeffs, ops, alpha, beta, chi_max, chi_sum, rel_tol);
  return write_train("rtt_pauli_apply", out, bond_out, cores_out, cap, n_out);
}

static rtt_status rtt_tt_combine_impl(int32_t n_trains, int32_t n_cores, const int32_t* bonds, const double* const* cores,
                          const double* coeffs, int32_t chi_max, double rel_tol, int32_t* bond_out,
                          double* cores_out, int64_t cap, int64_t* n_out) {
  g_err.clear();
  if (n_trains < 1 || !bonds || !cores || !coeffs) return fail(RTT_E_ARG, "rtt_tt_combine: no trains or null pointer");
  if (chi_max < 1 || !(rel_tol >= 0.0)) return fail(RTT_E_ARG, "rtt_tt_combine: chi_max %d, rel_tol %g", chi_max, rel_tol);
  std::vector<rtt_tt::Train> trains(n_trains);
  for (int m = 0; m < n_trains; ++m) {
    if (!isfinite(coeffs[m])) return fail(RTT_E_ARG, "rtt_tt_combine: coeffs[%d] is not finite", m);
    rtt_status st = read_train("rtt_tt_combine", n_cores, bonds + (size_t)m * (n_cores + 1), cores[m], trains[m]);
    if (st != RTT_OK) return st;
  }
  const rtt_tt::Train out = rtt_tt::combine(std::move(trains), coeffs, chi_max, rel_tol);
  return write_train("rtt_tt_combine", out, bond_out, cores_out, cap, n_out);
}

rtt_status rtt_tt_round(int32_t n_cores, const int32_t* bond, const double* cores, int32_t chi_max,
                        double rel_tol, int32_t* bond_out, double* cores_out, int64_t cap, int64_t* n_out) {
  return host_guard("rtt_tt_round", [&] {
    return rtt_tt_round_impl(n_cores, bond, cores, chi_max, rel_tol, bond_out, cores_out, cap, n_out);
  });
}

rtt_status rtt_tfim_power_step(int32_t n_spins, int32_t n_cores, const int32_t* pi, const int32_t* bond,
                               const double* cores, int32_t Lx, int32_t Ly, int32_t periodic, double J, double h,
                               double tau, int32_t chi_max, double rel_tol, int32_t* bond_out, double* cores_out,
                               int64_t cap, int64_t* n_out) {
  return host_guard("rtt_tfim_power_step", [&] {
    return rtt_tfim_power_step_impl(n_spins, n_cores, pi, bond, cores, Lx, Ly, periodic, J, h, tau, chi_max,
                                    rel_tol, bond_out, cores_out, cap, n_out);
  });
}

rtt_status rtt_pauli_apply(int32_t n_cores, const int32_t* bond, const double* cores, int32_t n_terms,
                           const double* coeffs, const uint8_t* ops, double alpha, double beta, int32_t chi_max,
                           int32_t chi_sum, double rel_tol, int32_t* bond_out, double* cores_out, int64_t cap,
                           int64_t* n_out) {
  return host_guard("rtt_pauli_apply", [&] {
    return rtt_pauli_apply_impl(n_cores, bond, cores, n_terms, coeffs, ops, alpha, beta, chi_max, chi_sum,
                                rel_tol, bond_out, cores_out, cap, n_out);
  });
}

rtt_status rtt_tt_combine(int32_t n_trains, int32_t n_cores, const int32_t* bonds, const double* const* cores,
                          const double* coeffs, int32_t chi_max, double rel_tol, int32_t* bond_out,
                          double* cores_out, int64_t cap, int64_t* n_out) {
  return host_guard("rtt_tt_combine", [&] {
    return rtt_tt_combine_impl(n_trains, n_cores, bonds, cores, coeffs, chi_max, rel_tol, bond_out, cores_out,
                               cap, n_out);
  });
}

static rtt_status rtt_batch_create_impl(int32_t n, const rtt_t* rtts, const rtt_ham_t* hams, const int32_t* walkers,
                                        uint64_t* const* spins, double* const* eloc, uint64_t seed, rtt_batch_t* out);
static rtt_status rtt_batch_autotune_impl(rtt_batch_t b, int32_t n_sweeps, int32_t reps, const char* cache_path,
                                          int32_t* choice, void* stream);
static rtt_status rtt_net_create_impl(int32_t Lx, int32_t Ly, const double* params, rtt_net_t* out);

rtt_status rtt_create(int32_t n_spins, int32_t n_cores, const int32_t* pi, const int32_t* bond,
                      const double* cores, int32_t dtype, rtt_t* out) {
  return host_guard("rtt_create", [&] { return rtt_create_impl(n_spins, n_cores, pi, bond, cores, dtype, out); });
}

rtt_status rtt_lincomb(int32_t n_terms, const rtt_t* terms, const double* coeffs, rtt_t* out) {
  return host_guard("rtt_lincomb", [&] { return rtt_lincomb_impl(n_terms, terms, coeffs, out); });
}

rtt_status rtt_tfim_create(int32_t Lx, int32_t Ly, int32_t periodic, double J, double h, rtt_ham_t* out) {
  return host_guard("rtt_tfim_create", [&] { return rtt_tfim_create_impl(Lx, Ly, periodic, J, h, out); });
}

rtt_status rtt_batch_create(int32_t n, const rtt_t* rtts, const rtt_ham_t* hams, const int32_t* walkers,
                            uint64_t* const* spins, double* const* eloc, uint64_t seed, rtt_batch_t* out) {
  return host_guard("rtt_batch_create", [&] { return rtt_batch_create_impl(n, rtts, hams, walkers, spins, eloc, seed, out); });
}

rtt_status rtt_batch_autotune(rtt_batch_t b, int32_t n_sweeps, int32_t reps, const char* cache_path,
                              int32_t* choice, void* stream) {
  return host_guard("rtt_batch_autotune", [&] { return rtt_batch_autotune_impl(b, n_sweeps, reps, cache_path, choice, stream); });
}

rtt_status rtt_net_create(int32_t Lx, int32_t Ly, const double* params, rtt_net_t* out) {
  return host_guard("rtt_net_create", [&] { return rtt_net_create_impl(Lx, Ly, params, out); });
}

rtt_status rtt_pair_sums(int32_t A, int32_t B, int32_t W, const double* x, const double* y, double* out,
                         void* stream) {
  g_err.clear();
  if (A < 1 || B < 1 || W < 1 || !x || !out) return fail(RTT_E_ARG, "rtt_pair_sums: bad argument");
  if (!y && B != 1) return fail(RTT_E_ARG, "rtt_pair_sums: row sums (y null) take B = 1");
  if ((int64_t)A * B > INT_MAX) return fail(RTT_E_ARG, "rtt_pair_sums: A * B too large");
  hipLaunchKernelGGL(rttk::pair_sums_kernel, dim3(A * B), dim3(256), 0, (hipStream_t)stream, B, W, x, y, out);
  HIPX(hipGetLastError());
  return RTT_OK;
}

rtt_status rtt_energy_reduce(int32_t n, const double* x, double* out, void* stream) {
  g_err.clear();
  if (n < 0 || (n > 0 && !x) || !out) return fail(RTT_E_ARG, "rtt_energy_reduce: bad argument");
  hipLaunchKernelGGL(rttk::reduce_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, n, x, out);
  HIPX(hipGetLastError());
  return RTT_OK;
}

}  // extern "C"

// ============================================================================
// batches
// ============================================================================
namespace {

// one bond class (dtype, padded bond) of a batch
struct BatchClass {
  int dtype = 0, chi = 0;
  int cg = 1, cg_max = 1;              // sampler walkers per block = 16 cg (autotuned)
  std::vector<int> members;
  std::vector<rttk::ChainArgs> chain;  // one descriptor per member
  std::vector<rttk::PassArgs> pass;    // forward and backward per member
  std::vector<int4> chain_items, pass_items;
  double chain_cost = 0, pass_cost = 0;
  size_t chain_lds = 0, pass_lds = 0;
  rttk::ChainArgs* d_chain = nullptr;
  rttk::PassArgs* d_pass = nullptr;
  int4* d_chain_items = nullptr;
  int4* d_pass_items = nullptr;
  int grid_chain = 1, grid_pass = 1;
  hipStream_t stream = nullptr;
};

}  // namespace

struct rtt_batch_s {
  int n = 0;
  uint64_t seed = 0;
  std::vector<rtt_s*> rtts;
  std::vector<rtt_ham_s*> hams;
  std::vector<int> W;
  std::vector<uint64_t*> spins;
  std::vector<double*> eloc;
  std::vector<float*> ws_f;      // per run: forward and backward cut vectors
  std::vector<int*> ws_i;        // per run: their exponents
  std::vector<BatchClass> classes;
  std::vector<rttk::CombineArgs> comb;
  std::vector<int4> comb_items;
  rttk::CombineArgs* d_comb = nullptr;
  int4* d_comb_items = nullptr;
  int* d_counters = nullptr;     // [2 * classes + 1]
  uint64_t* d_sweep0 = nullptr;
  int* d_red_n = nullptr;
  const double** d_red_x = nullptr;
  int concurrent = 0, occ = 1;   // launch shape
  int cus = 256;
  hipStream_t cap = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  std::vector<hipEvent_t> done;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_sweeps = -1;
  double* graph_esum = nullptr;
};

namespace {

// Sampler tile of a class: 16 walkers per block, or 32 (two column groups
// sharing every core fragment) at the bonds where that kernel fits in
// registers (at 64 and 256 the second group's operands spill).
constexpr bool batch_cg2(int chi) { return chi == 32 || chi == 128; }
template <class D, int CHI>
constexpr bool kBatchCG2 = batch_cg2(CHI);

template <class D, int CHI>
struct BatchL {
  static rtt_status run(BatchClass& c, int* counters, const uint64_t* sweep0, int phase, hipStream_t s) {
    auto kchain = rttk::chain_persistent<D, CHI, 1>;
    if constexpr (kBatchCG2<D, CHI>)
      if (c.cg == 2) kchain = rttk::chain_persistent<D, CHI, 2>;
    if (phase == 2) {  // before capture: allow the dynamic LDS sizes
      HIPX(hipFuncSetAttribute((const void*)kchain, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.chain_lds));
      HIPX(hipFuncSetAttribute((const void*)rttk::pass_persistent<D, CHI>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.pass_lds));
      return RTT_OK;
    }
    if (phase == 0) {
      if (c.chain_items.empty()) return RTT_OK;
      hipLaunchKernelGGL(kchain, dim3(c.grid_chain), dim3(rttk::ChainGeo<CHI, D>::NT), c.chain_lds, s, c.d_chain,
                         c.d_chain_items, (int)c.chain_items.size(), counters, sweep0);
    } else {
      if (c.pass_items.empty()) return RTT_OK;
      auto kfn = rttk::pass_persistent<D, CHI>;
      hipLaunchKernelGGL(kfn, dim3(c.grid_pass), dim3(256), c.pass_lds, s, c.d_pass, c.d_pass_items,
                         (int)c.pass_items.size(), counters);
    }
    HIPX(hipGetLastError());
    return RTT_OK;
  }
};

// persistent blocks per compute unit that the class's LDS allows
int lds_occupancy(size_t lds) { return std::max(1, std::min(4, (int)(kLdsLimit / std::max<size_t>(lds, 1)))); }

// Sampler work items of a class for cg column groups of 16 walkers per
// block: (member, block) pairs, members largest first; and the LDS the
// widest member needs.
void build_chain_items(const rtt_batch_s* b, BatchClass& c, int cg) {
  c.cg = cg;
  c.chain_items.clear();
  c.chain_lds = 0;
  for (int mi = 0; mi < (int)c.members.size(); ++mi) {
    const rtt_s* h = b->rtts[c.members[mi]];
    const int W = b->W[c.members[mi]];
    c.chain_lds = std::max(c.chain_lds, chain_lds_bytes(c.chi, h->T, h->L, h->nw, h->N, cg));
    for (int t = 0; t < (W + 16 * cg - 1) / (16 * cg); ++t) c.chain_items.push_back(make_int4(mi, t, 0, 0));
  }
}

rtt_status set_class_cg(rtt_batch_s* b, BatchClass& c, int cg) {
  build_chain_items(b, c, cg);
  if (c.d_chain_items) HIPX(hipFree(c.d_chain_items));
  c.d_chain_items = nullptr;
  return upload((void**)&c.d_chain_items, c.chain_items.data(), c.chain_items.size() * sizeof(int4));
}

void size_grids(rtt_batch_s* b) {
  double tot_c = 0, tot_p = 0;
  for (auto& c : b->classes) { tot_c += c.chain_cost; tot_p += c.pass_cost; }
  for (auto& c : b->classes) {
    const int occ_c = std::min(b->occ, lds_occupancy(c.chain_lds));
    const int occ_p = std::min(b->occ, lds_occupancy(c.pass_lds));
    int gc = b->cus * occ_c, gp = b->cus * occ_p;
    if (b->concurrent) {  // compute units shared in proportion to the work
      gc = (int)std::lround(gc * (tot_c > 0 ? c.chain_cost / tot_c : 0.0));
      gp = (int)std::lround(gp * (tot_p > 0 ? c.pass_cost / tot_p : 0.0));
    }
    c.grid_chain = std::max(1, std::min(gc, (int)c.chain_items.size()));
    c.grid_pass = std::max(1, std::min(gp, (int)c.pass_items.size()));
  }
}

rtt_status record_step(rtt_batch_s* b, int n_sweeps, double* esum, hipStream_t s) {
  const int nc = (int)b->classes.size();
  hipLaunchKernelGGL(rttk::fill_int, dim3(1), dim3(64), 0, s, b->d_counters, 2 * nc + 1, 0);
  HIPX(hipGetLastError());
  for (int phase = 0; phase < 2; ++phase) {
    if (phase == 0 && n_sweeps == 0) continue;
    if (b->concurrent) {
      HIPX(hipEventRecord(b->fork, s));
      for (int ci = 0; ci < nc; ++ci) {
        BatchClass& c = b->classes[ci];
        HIPX(hipStreamWaitEvent(c.stream, b->fork, 0));
        rtt_status st = dispatch<BatchL>(c.dtype, c.chi, c, b->d_counters + 2 * ci + phase, b->d_sweep0, phase, c.stream);
        if (st != RTT_OK) return st;
        HIPX(hipEventRecord(b->done[ci], c.stream));
      }
      for (int ci = 0; ci < nc; ++ci) HIPX(hipStreamWaitEvent(s, b->done[ci], 0));
    } else {
      for (int ci = 0; ci < nc; ++ci) {
        BatchClass& c = b->classes[ci];
        rtt_status st = dispatch<BatchL>(c.dtype, c.chi, c, b->d_counters + 2 * ci + phase, b->d_sweep0, phase, s);
        if (st != RTT_OK) return st;
      }
    }
  }
  hipLaunchKernelGGL(rttk::combine_persistent, dim3(std::min<int>(b->cus * 4, (int)b->comb_items.size())),
                     dim3(256), 0, s, b->d_comb, b->d_comb_items, (int)b->comb_items.size(),
                     b->d_counters + 2 * nc);
  HIPX(hipGetLastError());
  if (esum) {
    hipLaunchKernelGGL(rttk::reduce_many, dim3(b->n), dim3(256), 0, s, b->d_red_n, b->d_red_x, esum);
    HIPX(hipGetLastError());
  }
  hipLaunchKernelGGL(rttk::advance_u64, dim3(1), dim3(64), 0, s, b->d_sweep0, (uint64_t)n_sweeps);
  HIPX(hipGetLastError());
  return RTT_OK;
}

rtt_status set_sweeps(rtt_batch_s* b, int n_sweeps) {
  for (auto& c : b->classes) {
    for (auto& d : c.chain) d.n_sweeps = n_sweeps;
    HIPX(hipMemcpy(c.d_chain, c.chain.data(), c.chain.size() * sizeof(rttk::ChainArgs), hipMemcpyHostToDevice));
  }
  return RTT_OK;
}

rtt_status capture(rtt_batch_s* b, int n_sweeps, double* esum) {
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  rtt_status st = set_sweeps(b, n_sweeps);
  if (st != RTT_OK) return st;
  size_grids(b);
  for (auto& c : b->classes) {
    st = dispatch<BatchL>(c.dtype, c.chi, c, (int*)nullptr, (const uint64_t*)nullptr, 2, b->cap);
    if (st != RTT_OK) return st;
  }
  HIPX(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  st = record_step(b, n_sweeps, esum, b->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (st != RTT_OK) { if (g) (void)hipGraphDestroy(g); return st; }
  if (e != hipSuccess) return fail(RTT_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
  b->graph = g;
  HIPX(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  b->graph_sweeps = n_sweeps;
  b->graph_esum = esum;
  return RTT_OK;
}

void free_batch(rtt_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto& c : b->classes) {
    for (void* p : {(void*)c.d_chain, (void*)c.d_pass, (void*)c.d_chain_items, (void*)c.d_pass_items})
      if (p) (void)hipFree(p);
    if (c.stream) (void)hipStreamDestroy(c.stream);
  }
  for (void* p : {(void*)b->d_comb, (void*)b->d_comb_items, (void*)b->d_counters, (void*)b->d_sweep0,
                  (void*)b->d_red_n, (void*)b->d_red_x})
    if (p) (void)hipFree(p);
  for (auto p : b->ws_f) if (p) (void)hipFree(p);
  for (auto p : b->ws_i) if (p) (void)hipFree(p);
  for (auto e : b->done) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->join) (void)hipEventDestroy(b->join);
  if (b->cap) (void)hipStreamDestroy(b->cap);
}

std::string batch_signature(const rtt_batch_s* b) {
  std::string sig;
  char buf[96];
  for (int i = 0; i < b->n; ++i) {
    snprintf(buf, sizeof buf, "%d:%d:%d:%d:%d;", b->rtts[i]->dtype, b->rtts[i]->chi, b->rtts[i]->L,
             b->rtts[i]->N, b->W[i]);
    sig += buf;
  }
  // FNV-1a of the description keeps cache keys short
  uint64_t h = 1469598103934665603ull;
  for (char ch : sig) { h ^= (unsigned char)ch; h *= 1099511628211ull; }
  snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
  return buf;
}

}  // namespace

extern "C" {

static rtt_status rtt_batch_create_impl(int32_t n, const rtt_t* rtts, const rtt_ham_t* hams, const int32_t* walkers,
                            uint64_t* const* spins, double* const* eloc, uint64_t seed, rtt_batch_t* out) {
  g_err.clear();
  if (!out) return fail(RTT_E_ARG, "rtt_batch_create: out is null");
  *out = nullptr;
  if (n < 1 || !rtts || !hams || !walkers || !spins || !eloc) return fail(RTT_E_ARG, "rtt_batch_create: bad argument");
  for (int i = 0; i < n; ++i) {
    if (!rtts[i] || !hams[i] || walkers[i] < 1 || !spins[i] || !eloc[i])
      return fail(RTT_E_ARG, "rtt_batch_create: run %d has a null handle, buffer or no walkers", i);
    if (hams[i]->Lx * hams[i]->Ly != rtts[i]->N)
      return fail(RTT_E_ARG, "rtt_batch_create: run %d: lattice and RTT sizes differ", i);
  }
  rtt_batch_s* b = new rtt_batch_s;
  b->n = n;
  b->seed = seed;
  b->rtts.assign(rtts, rtts + n);
  b->hams.assign(hams, hams + n);
  b->W.assign(walkers, walkers + n);
  b->spins.assign(spins, spins + n);
  b->eloc.assign(eloc, eloc + n);
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) b->cus = prop.multiProcessorCount;

  auto cleanup = [&](rtt_status st) { free_batch(b); delete b; return st; };
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j)
      if (b->rtts[i] == b->rtts[j] || b->spins[i] == b->spins[j] || b->eloc[i] == b->eloc[j]) {
        delete b;
        return fail(RTT_E_ARG, "rtt_batch_create: runs %d and %d share an RTT handle or a buffer", j, i);
      }
  // the batch's own cut-vector workspace for every run
  b->ws_f.assign(n, nullptr);
  b->ws_i.assign(n, nullptr);
  for (int i = 0; i < n; ++i) {
    const rtt_s* h = b->rtts[i];
    const size_t rows = (size_t)h->T * h->sched.ng * b->W[i] * h->sched.nslot;
    if (hipMalloc(&b->ws_f[i], 2 * rows * h->chi * 4) != hipSuccess ||
        hipMalloc(&b->ws_i[i], 2 * rows * 4) != hipSuccess)
      return cleanup(fail(RTT_E_OOM, "rtt_batch_create: workspace for run %d", i));
  }
  auto ws_u = [&](int i) { return b->ws_f[i]; };
  auto ws_v = [&](int i) {
    const rtt_s* h = b->rtts[i];
    return b->ws_f[i] + (size_t)h->T * h->sched.ng * b->W[i] * h->sched.nslot * h->chi;
  };
  auto ws_ue = [&](int i) { return b->ws_i[i]; };
  auto ws_ve = [&](int i) {
    const rtt_s* h = b->rtts[i];
    return b->ws_i[i] + (size_t)h->T * h->sched.ng * b->W[i] * h->sched.nslot;
  };
  // group runs by (dtype, padded bond); order members by work, largest first
  for (int i = 0; i < n; ++i) {
    const rtt_s* h = b->rtts[i];
    int ci = -1;
    for (int c = 0; c < (int)b->classes.size(); ++c)
      if (b->classes[c].dtype == h->dtype && b->classes[c].chi == h->chi) ci = c;
    if (ci < 0) {
      b->classes.emplace_back();
      ci = (int)b->classes.size() - 1;
      b->classes[ci].dtype = h->dtype;
      b->classes[ci].chi = h->chi;
    }
    b->classes[ci].members.push_back(i);
  }
  for (auto& c : b->classes) {
    const double chi2 = (double)c.chi * c.chi;
    std::vector<std::pair<double, int>> order;
    for (int i : c.members) {
      const rtt_s* h = b->rtts[i];
      const double rows = (double)h->sched.cost * 16;
      order.push_back({rows * chi2 * h->T, i});
    }
    std::sort(order.begin(), order.end(), [](auto& x, auto& y) { return x.first > y.first; });
    c.members.clear();
    for (auto& o : order) c.members.push_back(o.second);
    for (int mi = 0; mi < (int)c.members.size(); ++mi) {
      const int i = c.members[mi];
      rtt_s* h = b->rtts[i];
      const int W = b->W[i];
      rttk::ChainArgs ca{};
      ca.cores = h->d_fwd; ca.cores_bwd = h->d_bwd; ca.cesum = h->d_cesum; ca.rmask = h->d_rmask; ca.pi = h->d_pi;
      ca.order = h->d_order; ca.first = h->d_first; ca.coeffs = h->d_coeffs;
      ca.T = h->T; ca.L = h->L; ca.N = h->N; ca.nw = h->nw; ca.LW = (h->L + 63) / 64; ca.W = W;
      ca.spins = b->spins[i]; ca.seed = seed; ca.rstream = (uint64_t)i; ca.mode = 1;
      c.chain.push_back(ca);

      rttk::PassArgs pa{};
      pa.core_exp = h->d_cexp; pa.nslot = h->sched.nslot; pa.L = h->L; pa.nw = h->nw; pa.W = W;
      pa.spins = b->spins[i];
      pa.ng = h->sched.ng;
      pa.cores = h->d_fwd; pa.sched = h->d_sf; pa.gsteps = h->d_fgs;
      pa.out_vec = ws_u(i); pa.out_exp = ws_ue(i);
      c.pass.push_back(pa);
      pa.cores = h->d_bwd; pa.sched = h->d_sb; pa.gsteps = h->d_bgs;
      pa.out_vec = ws_v(i); pa.out_exp = ws_ve(i);
      c.pass.push_back(pa);
      c.pass_lds = std::max(c.pass_lds, pass_lds_bytes(c.chi, h->sched.nslot, h->nw, h->dtype));
      // sweep cost ~ (L + sum_j (L - first_j)) row-steps per walker tile
      double sweep_rows = h->L;
      for (int j = 0; j < h->N; ++j) if (h->first[j] >= 0) sweep_rows += h->L - h->first[j];
      c.chain_cost += sweep_rows * h->T * ((W + 15) / 16) * 16 * (double)c.chi * c.chi;
      const int wpb = 4 / rttk_wpw(c.chi);
      c.pass_cost += (double)h->sched.cost * 16 * h->T * W * (double)c.chi * c.chi;

      for (int dir = 0; dir < 2; ++dir)
        for (int ty = 0; ty < h->T * h->sched.ng; ++ty)
          for (int bx = 0; bx < (W + wpb - 1) / wpb; ++bx) c.pass_items.push_back(make_int4(2 * mi + dir, bx, ty, 0));
    }
    // sampler tiles: 16 walkers per block; 32 allowed where every member's
    // state fits on chip in the same layout (same results, bit for bit)
    c.cg_max = batch_cg2(c.chi) ? 2 : 1;
    for (int i : c.members) {
      const rtt_s* h = b->rtts[i];
      const int LW = (h->L + 63) / 64;
      const rttk::ChainLayout l1(c.chi, h->T, LW, h->nw, 1, 0, h->N), l2(c.chi, h->T, LW, h->nw, 2, 0, h->N);
      if (l2.seq != l1.seq || (size_t)l2.total > kLdsLimit) c.cg_max = 1;
    }
    const char* tile = getenv("RTT_BATCH_TILE");
    build_chain_items(b, c, (tile && atoi(tile) == 32 && c.cg_max == 2) ? 2 : 1);
    rtt_status st;
    if ((st = upload((void**)&c.d_chain, c.chain.data(), c.chain.size() * sizeof(rttk::ChainArgs))) != RTT_OK) return cleanup(st);
    if ((st = upload((void**)&c.d_pass, c.pass.data(), c.pass.size() * sizeof(rttk::PassArgs))) != RTT_OK) return cleanup(st);
    if ((st = upload((void**)&c.d_chain_items, c.chain_items.data(), c.chain_items.size() * sizeof(int4))) != RTT_OK) return cleanup(st);
    if ((st = upload((void**)&c.d_pass_items, c.pass_items.data(), c.pass_items.size() * sizeof(int4))) != RTT_OK) return cleanup(st);
    if (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess) return cleanup(fail(RTT_E_HIP, "stream create"));
  }
  // combine descriptors: one per run; items of 4 walkers, biggest runs first
  std::vector<int> by_size(n);
  for (int i = 0; i < n; ++i) by_size[i] = i;
  std::sort(by_size.begin(), by_size.end(), [&](int x, int y) { return b->W[x] * b->rtts[x]->N > b->W[y] * b->rtts[y]->N; });
  for (int i = 0; i < n; ++i) {
    rtt_s* h = b->rtts[i];
    rttk::CombineArgs ca{};
    ca.u = ws_u(i); ca.ue = ws_ue(i); ca.v = ws_v(i); ca.ve = ws_ve(i);
    ca.nsf = h->sched.nslot; ca.nsb = h->sched.nslot; ca.chi = h->chi; ca.T = h->T; ca.W = b->W[i];
    ca.N = h->N; ca.nw = h->nw; ca.fslot = h->d_fslot; ca.bslot = h->d_bslot; ca.coeffs = h->d_coeffs;
    ca.ng = h->sched.ng; ca.grp = h->d_grp;
    ca.spins = b->spins[i]; ca.bonds = b->hams[i]->d_bonds; ca.nbonds = b->hams[i]->nb;
    ca.J = b->hams[i]->J; ca.h = b->hams[i]->h; ca.eloc = b->eloc[i];
    b->comb.push_back(ca);
  }
  for (int i : by_size)
    for (int bx = 0; bx < (b->W[i] + 3) / 4; ++bx) b->comb_items.push_back(make_int4(i, bx, 0, 0));
  rtt_status st;
  if ((st = upload((void**)&b->d_comb, b->comb.data(), b->comb.size() * sizeof(rttk::CombineArgs))) != RTT_OK) return cleanup(st);
  if ((st = upload((void**)&b->d_comb_items, b->comb_items.data(), b->comb_items.size() * sizeof(int4))) != RTT_OK) return cleanup(st);
  std::vector<int> zeros(2 * b->classes.size() + 1, 0);
  if ((st = upload((void**)&b->d_counters, zeros.data(), zeros.size() * 4)) != RTT_OK) return cleanup(st);
  uint64_t z64 = 0;
  if ((st = upload((void**)&b->d_sweep0, &z64, 8)) != RTT_OK) return cleanup(st);
  std::vector<const double*> xs(b->eloc.begin(), b->eloc.end());
  if ((st = upload((void**)&b->d_red_n, b->W.data(), n * 4)) != RTT_OK) return cleanup(st);
  if ((st = upload((void**)&b->d_red_x, xs.data(), n * sizeof(double*))) != RTT_OK) return cleanup(st);
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) return cleanup(fail(RTT_E_HIP, "stream create"));
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) return cleanup(fail(RTT_E_HIP, "event create"));
  if (hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess) return cleanup(fail(RTT_E_HIP, "event create"));
  b->done.resize(b->classes.size());
  for (auto& e : b->done)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return cleanup(fail(RTT_E_HIP, "event create"));
  *out = b;
  return RTT_OK;
}

rtt_status rtt_batch_step(rtt_batch_t b, int32_t n_sweeps, double* esum, void* stream) {
  g_err.clear();
  if (!b) return fail(RTT_E_ARG, "rtt_batch_step: null batch");
  if (n_sweeps < 0) return fail(RTT_E_ARG, "rtt_batch_step: n_sweeps < 0");
  if (!b->exec || b->graph_sweeps != n_sweeps || b->graph_esum != esum) {
    HIPX(hipDeviceSynchronize());
    rtt_status st = capture(b, n_sweeps, esum);
    if (st != RTT_OK) return st;
  }
  HIPX(hipGraphLaunch(b->exec, (hipStream_t)stream));
  return RTT_OK;
}

static rtt_status rtt_batch_autotune_impl(rtt_batch_t b, int32_t n_sweeps, int32_t reps, const char* cache_path,
                              int32_t* choice, void* stream) {
  g_err.clear();
  if (!b || reps < 1 || n_sweeps < 0) return fail(RTT_E_ARG, "rtt_batch_autotune: bad argument");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIPX(hipEventCreate(&e0));
  HIPX(hipEventCreate(&e1));
  // one timed trial of the current shape and tiles: a capture, one warm-up
  // step, reps timed steps
  auto trial = [&](float& ms) -> rtt_status {
    HIPX(hipDeviceSynchronize());
    rtt_status st = capture(b, n_sweeps, nullptr);
    if (st != RTT_OK) return st;
    HIPX(hipGraphLaunch(b->exec, s));
    HIPX(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) HIPX(hipGraphLaunch(b->exec, s));
    HIPX(hipEventRecord(e1, s));
    HIPX(hipEventSynchronize(e1));
    HIPX(hipEventElapsedTime(&ms, e0, e1));
    return RTT_OK;
  };
  // launch shape: concurrency of the classes and persistent blocks per CU
  float best = 1e30f;
  int best_conc = 0, best_occ = 1;
  for (int conc = 0; conc < 2; ++conc)
    for (int occ = 1; occ <= 4; ++occ) {
      b->concurrent = conc;
      b->occ = occ;
      float ms = 0.f;
      rtt_status st = trial(ms);
      if (st != RTT_OK) return st;
      if (ms < best) { best = ms; best_conc = conc; best_occ = occ; }
    }
  b->concurrent = best_conc;
  b->occ = best_occ;
  // tiles: per class, the sampler's walkers per block (16, or 32 sharing
  // every core fragment), one class at a time with the others as chosen
  int trials = 8;
  for (auto& c : b->classes) {
    if (c.cg_max < 2) continue;
    const int other = c.cg == 2 ? 1 : 2;
    const int keep = c.cg;
    rtt_status st = set_class_cg(b, c, other);
    if (st != RTT_OK) return st;
    float ms = 0.f;
    if ((st = trial(ms)) != RTT_OK) return st;
    ++trials;
    if (ms < best) best = ms;
    else if ((st = set_class_cg(b, c, keep)) != RTT_OK) return st;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  if (choice) { choice[0] = best_conc; choice[1] = best_occ; }
  if (cache_path) {
    // append one JSON object per line: signature, choice, time per step
    std::string tiles;
    char buf[96];
    for (size_t ci = 0; ci < b->classes.size(); ++ci) {
      snprintf(buf, sizeof buf, "%s{\"dtype\": %d, \"bond\": %d, \"sampler_walkers_per_block\": %d}", ci ? ", " : "",
               b->classes[ci].dtype, b->classes[ci].chi, 16 * b->classes[ci].cg);
      tiles += buf;
    }
    FILE* f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "{\"batch\": \"%s\", \"runs\": %d, \"sweeps\": %d, \"concurrent\": %d, \"blocks_per_cu\": %d, "
              "\"classes\": [%s], \"trials\": %d, \"ms_per_step\": %.4f}\n",
              batch_signature(b).c_str(), b->n, n_sweeps, best_conc, best_occ, tiles.c_str(), trials, best / reps);
      fclose(f);
    }
  }
  return RTT_OK;
}

rtt_status rtt_batch_destroy(rtt_batch_t b) {
  if (!b) return RTT_OK;
  HIPX(hipDeviceSynchronize());
  free_batch(b);
  delete b;
  return RTT_OK;
}

}  // extern "C"

// ============================================================================
// learned proposal
// ============================================================================
struct rtt_net_s {
  int Lx = 0, Ly = 0, N = 0, nw = 0;
  float* d_master = nullptr;
  float* d_infer = nullptr;
  uint16_t* d_wpk = nullptr;  // middle layers packed for the matrix cores
  float* d_m = nullptr;
  float* d_v = nullptr;
  float* d_grad = nullptr;
  double* d_baseline = nullptr;
  int t = 0;
  int W_ws = 0, B_ws = 0;
  uint64_t* d_prop = nullptr;
  int* d_moves = nullptr;
  double* d_lqf = nullptr;
  double* d_lqr = nullptr;
  double* d_la = nullptr;
  int8_t* d_sg = nullptr;
  int32_t* d_st = nullptr;
  float* d_partial = nullptr;
};

namespace {

void free_net(rtt_net_s* n) {
  for (void* p : {(void*)n->d_master, (void*)n->d_infer, (void*)n->d_wpk, (void*)n->d_m, (void*)n->d_v,
                  (void*)n->d_grad, (void*)n->d_baseline})
    if (p) (void)hipFree(p);
  bool any = false;
  for (void* p : {(void*)n->d_prop, (void*)n->d_moves, (void*)n->d_lqf, (void*)n->d_lqr, (void*)n->d_la,
                  (void*)n->d_sg, (void*)n->d_st, (void*)n->d_partial})
    if (p) { (void)hipFreeAsync(p, nullptr); any = true; }
  if (any) (void)hipDeviceSynchronize();
}

rtt_status net_ws(rtt_net_s* n, int W, hipStream_t s) {
  if (W <= n->W_ws) return RTT_OK;
  n->W_ws = 0;
  rtt_status st;
  if ((st = grow_async((void**)&n->d_prop, (size_t)W * n->nw * 8, s)) != RTT_OK) return st;
  if ((st = grow_async((void**)&n->d_moves, (size_t)W * 4, s)) != RTT_OK) return st;
  if ((st = grow_async((void**)&n->d_lqf, (size_t)W * 8, s)) != RTT_OK) return st;
  if ((st = grow_async((void**)&n->d_lqr, (size_t)W * 8, s)) != RTT_OK) return st;
  if ((st = grow_async((void**)&n->d_la, (size_t)W * 8, s)) != RTT_OK) return st;
  if ((st = grow_async((void**)&n->d_sg, (size_t)W, s)) != RTT_OK) return st;
  if ((st = grow_async((void**)&n->d_st, (size_t)W * 4, s)) != RTT_OK) return st;
  n->W_ws = W;
  return RTT_OK;
}

rtt_status net_set_lds(const void* f, size_t bytes) {
  HIPX(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return RTT_OK;
}

constexpr int kNetSlices = 32;  // first-stage slices of the gradient sum over samples

rtt_status net_grad_launch(rtt_net_s* n, int B, const uint64_t* spins, const int32_t* moves,
                           const float* accept_prob, float* grad, hipStream_t s) {
  if (B > n->B_ws) {
    n->B_ws = 0;
    // per-sample gradients, then room for the slice sums of the reduction
    rtt_status st = grow_async((void**)&n->d_partial, (size_t)(B + kNetSlices) * rttk::kNetParams * 4, s);
    if (st != RTT_OK) return st;
    n->B_ws = B;
  }
  rttk::NetGradArgs ga{};
  ga.P = n->d_infer; ga.Lx = n->Lx; ga.Ly = n->Ly; ga.nw = n->nw; ga.B = B;
  ga.spins = spins; ga.moves = moves; ga.accept_prob = accept_prob; ga.baseline = n->d_baseline;
  ga.partial = n->d_partial;
  const size_t lds = rttk::net_grad_lds_bytes(n->N);
  rtt_status st = net_set_lds((const void*)rttk::net_grad_kernel, lds);
  if (st != RTT_OK) return st;
  hipLaunchKernelGGL(rttk::net_grad_kernel, dim3(B), dim3(256), lds, s, ga);
  HIPX(hipGetLastError());
  const int S = std::min(B, kNetSlices);
  float* slices = n->d_partial + (size_t)B * rttk::kNetParams;
  hipLaunchKernelGGL(rttk::net_reduce_slices_kernel, dim3((rttk::kNetParams + 255) / 256, S), dim3(256), 0, s,
                     n->d_partial, B, S, slices);
  HIPX(hipGetLastError());
  hipLaunchKernelGGL(rttk::net_reduce_kernel, dim3((rttk::kNetParams + 255) / 256), dim3(256), 0, s,
                     slices, S, grad);
  HIPX(hipGetLastError());
  return RTT_OK;
}

}  // namespace

extern "C" {

static rtt_status rtt_net_create_impl(int32_t Lx, int32_t Ly, const double* params, rtt_net_t* out) {
  g_err.clear();
  if (!out) return fail(RTT_E_ARG, "rtt_net_create: out is null");
  *out = nullptr;
  if (Lx < 3 || Ly < 3 || Lx * Ly > 256) return fail(RTT_E_ARG, "rtt_net_create: lattice %dx%d (need sides >= 3, <= 256 sites)", Lx, Ly);
  if (!params) return fail(RTT_E_ARG, "rtt_net_create: params is null");
  std::vector<float> m(rttk::kNetParams), inf(rttk::kNetParams);
  for (int p = 0; p < rttk::kNetParams; ++p) {
    if (!isfinite(params[p])) return fail(RTT_E_ARG, "rtt_net_create: parameter %d not finite", p);
    m[p] = (float)params[p];
    inf[p] = (float)bf16_value(bf16_bits_rne(m[p]));
  }
  rtt_net_s* n = new rtt_net_s;
  n->Lx = Lx; n->Ly = Ly; n->N = Lx * Ly; n->nw = (n->N + 63) / 64;
  std::vector<float> zeros(rttk::kNetParams, 0.f);
  // the middle layers' weights as [layer][tap][co][ci] BF16 bits
  std::vector<uint16_t> pk(rttk::kNetPacked);
  for (int p = 0; p < rttk::kNetPacked; ++p) {
    const int layer = p / (9 * rttk::kNetC * rttk::kNetC), r = p % (9 * rttk::kNetC * rttk::kNetC);
    const int t = r / (rttk::kNetC * rttk::kNetC), co = (r / rttk::kNetC) % rttk::kNetC, ci = r % rttk::kNetC;
    pk[p] = bf16_bits_rne(inf[(layer == 0 ? rttk::oW2 : rttk::oW3) + (co * rttk::kNetC + ci) * 9 + t]);
  }
  double zb = 0.0;
  rtt_status st;
  if ((st = upload((void**)&n->d_master, m.data(), m.size() * 4)) != RTT_OK ||
      (st = upload((void**)&n->d_infer, inf.data(), inf.size() * 4)) != RTT_OK ||
      (st = upload((void**)&n->d_wpk, pk.data(), pk.size() * 2)) != RTT_OK ||
      (st = upload((void**)&n->d_m, zeros.data(), zeros.size() * 4)) != RTT_OK ||
      (st = upload((void**)&n->d_v, zeros.data(), zeros.size() * 4)) != RTT_OK ||
      (st = upload((void**)&n->d_grad, zeros.data(), zeros.size() * 4)) != RTT_OK ||
      (st = upload((void**)&n->d_baseline, &zb, 8)) != RTT_OK) {
    free_net(n);
    delete n;
    return st;
  }
  *out = n;
  return RTT_OK;
}

rtt_status rtt_net_destroy(rtt_net_t n) {
  if (!n) return RTT_OK;
  HIPX(hipDeviceSynchronize());
  free_net(n);
  delete n;
  return RTT_OK;
}

rtt_status rtt_net_get_params(rtt_net_t n, int32_t which, double* out) {
  g_err.clear();
  if (!n || !out || which < 0 || which > 1) return fail(RTT_E_ARG, "rtt_net_get_params: bad argument");
  std::vector<float> h(rttk::kNetParams);
  HIPX(hipDeviceSynchronize());
  HIPX(hipMemcpy(h.data(), which == 0 ? n->d_master : n->d_infer, h.size() * 4, hipMemcpyDeviceToHost));
  for (int p = 0; p < rttk::kNetParams; ++p) out[p] = h[p];
  return RTT_OK;
}

rtt_status rtt_net_forward(rtt_net_t n, int32_t W, const uint64_t* spins, float* out, void* stream) {
  g_err.clear();
  if (!n || W < 1 || !spins || !out) return fail(RTT_E_ARG, "rtt_net_forward: bad argument");
  rttk::NetMoveArgs a{};
  a.P = n->d_infer; a.wpk = n->d_wpk; a.Lx = n->Lx; a.Ly = n->Ly; a.nw = n->nw; a.W = W; a.spins = spins;
  a.out = out;
  const size_t lds = rttk::net_fwd_lds_bytes(n->N);
  rtt_status st = net_set_lds((const void*)rttk::net_forward_kernel, lds);
  if (st != RTT_OK) return st;
  hipLaunchKernelGGL(rttk::net_forward_kernel, dim3(W), dim3(256), lds, (hipStream_t)stream, a);
  HIPX(hipGetLastError());
  return RTT_OK;
}

rtt_status rtt_mh_learned_step(rtt_t h, rtt_net_t n, int32_t W, uint64_t* spins, double* logabs,
                               int8_t* sign, uint64_t seed, uint64_t rng_stream, uint64_t step,
                               int32_t* moves, float* accept_prob, uint64_t* before,
                               uint32_t* accepts, int32_t* status, void* stream) {
  g_err.clear();
  if (check_handle(h) != RTT_OK) return RTT_E_ARG;
  if (!n || W < 1 || !spins || !logabs || !sign) return fail(RTT_E_ARG, "rtt_mh_learned_step: bad argument");
  if (n->N != h->N) return fail(RTT_E_ARG, "rtt_mh_learned_step: network has %d sites, RTT %d spins", n->N, h->N);
  hipStream_t s = (hipStream_t)stream;
  rtt_status st = net_ws(n, W, s);
  if (st != RTT_OK) return st;
  rttk::NetMoveArgs a{};
  a.P = n->d_infer; a.wpk = n->d_wpk; a.Lx = n->Lx; a.Ly = n->Ly; a.nw = n->nw; a.W = W; a.spins = spins;
  a.prop = n->d_prop; a.moves = moves ? moves : n->d_moves; a.lqf = n->d_lqf; a.lqr = n->d_lqr;
  a.seed = seed; a.rstream = rng_stream; a.step = step; a.before = before;
  const size_t lds = rttk::net_fwd_lds_bytes(n->N);
  if ((st = net_set_lds((const void*)rttk::net_propose_kernel, lds)) != RTT_OK) return st;
  if ((st = net_set_lds((const void*)rttk::net_reverse_kernel, lds)) != RTT_OK) return st;
  hipLaunchKernelGGL(rttk::net_propose_kernel, dim3(W), dim3(256), lds, s, a);
  HIPX(hipGetLastError());
  hipLaunchKernelGGL(rttk::net_reverse_kernel, dim3(W), dim3(256), lds, s, a);
  HIPX(hipGetLastError());
  st = chain_common(h, W, n->d_prop, n->d_la, n->d_sg, 0, 0, 0, 0, nullptr, n->d_st, 0, stream);
  if (st != RTT_OK) return st;
  rttk::NetAcceptArgs c{};
  c.W = W; c.nw = n->nw; c.spins = spins; c.prop = n->d_prop; c.logabs = logabs; c.sign = sign;
  c.la_new = n->d_la; c.sg_new = n->d_sg; c.st_new = n->d_st; c.lqf = n->d_lqf; c.lqr = n->d_lqr;
  c.moves = a.moves; c.accept_prob = accept_prob; c.accepts = accepts; c.status = status;
  c.seed = seed; c.rstream = rng_stream; c.step = step;
  hipLaunchKernelGGL(rttk::net_accept_kernel, dim3((W + 255) / 256), dim3(256), 0, s, c);
  HIPX(hipGetLastError());
  return RTT_OK;
}

rtt_status rtt_net_grad(rtt_net_t n, int32_t B, const uint64_t* spins, const int32_t* moves,
                        const float* accept_prob, float* grad, void* stream) {
  g_err.clear();
  if (!n || B < 1 || !spins || !moves || !accept_prob || !grad) return fail(RTT_E_ARG, "rtt_net_grad: bad argument");
  return net_grad_launch(n, B, spins, moves, accept_prob, grad, (hipStream_t)stream);
}

rtt_status rtt_net_train(rtt_net_t n, int32_t B, const uint64_t* spins, const int32_t* moves,
                         const float* accept_prob, float lr, float beta1, float beta2, float eps,
                         void* stream) {
  g_err.clear();
  if (!n || B < 1 || !spins || !moves || !accept_prob) return fail(RTT_E_ARG, "rtt_net_train: bad argument");
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(RTT_E_ARG, "rtt_net_train: bad optimiser constants");
  hipStream_t s = (hipStream_t)stream;
  rtt_status st = net_grad_launch(n, B, spins, moves, accept_prob, n->d_grad, s);
  if (st != RTT_OK) return st;
  hipLaunchKernelGGL(rttk::net_baseline_kernel, dim3(1), dim3(256), 0, s, accept_prob, moves, B, n->d_baseline);
  HIPX(hipGetLastError());
  n->t += 1;
  hipLaunchKernelGGL(rttk::net_adam_kernel, dim3((rttk::kNetParams + 255) / 256), dim3(256), 0, s, n->d_master,
                     n->d_infer, n->d_m, n->d_v, n->d_grad, lr, beta1, beta2, eps, n->t);
  HIPX(hipGetLastError());
  hipLaunchKernelGGL(rttk::net_pack_kernel, dim3((rttk::kNetPacked + 255) / 256), dim3(256), 0, s, n->d_infer,
                     n->d_wpk);
  HIPX(hipGetLastError());
  return RTT_OK;
}

}  // extern "C"
