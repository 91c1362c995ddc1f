// Host tensor-train algebra for the replica-space power method (FP64).
//
// A train of L cores; core k is [2][a_k][a_{k+1}] row-major (a_0 = a_L = 1).
//   * Pauli strings in replica space act as rank-1 operators: X swaps the two
//     slices of a core, Z changes the sign of slice 1 (Sec. 2.2.3: X on a
//     spin acts on every replica, Z on one replica of the spin's choice).
//   * The sum of two trains has block-diagonal interior cores.
//   * Rounding (compression): right-to-left orthogonalisation by Householder
//     QR, then left-to-right truncated SVDs (one-sided Jacobi), keeping at
//     most chi_max singular values and none below rel_tol times the largest.
//   * A power step of the TFIM (Sec. 3.1): phi - tau H-bar phi, the terms of
//     H-bar phi summed two by two with a rounding after each sum.
#pragma once
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <new>
#include <thread>
#include <vector>

namespace rtt_tt {

struct Train {
  std::vector<int> bond;                 // L + 1
  std::vector<std::vector<double>> core;  // L cores, [2][a][b]
  int L() const { return (int)core.size(); }
  double& at(int k, int s, int i, int j) { return core[k][((size_t)s * bond[k] + i) * bond[k + 1] + j]; }
  double at(int k, int s, int i, int j) const { return core[k][((size_t)s * bond[k] + i) * bond[k + 1] + j]; }
};

// Scratch buffers of one thread, grown on demand and reused: rounding a long
// train of small cores would otherwise spend its time in the allocator.
struct Work {
  std::vector<double> W, Q, R, V, U, Vs, S, nrm, hv, betas, a, b;
  std::vector<int> ord;
};
inline Work& work() {
  thread_local Work w;
  return w;
}
inline double* grow(std::vector<double>& v, size_t n) {
  if (v.size() < n) v.resize(n);
  return v.data();
}

// frexp exponent of the largest |x_i| (0 for an all-zero array)
inline int max_exponent(size_t n, const double* x) {
  double mx = 0.0;
  for (size_t i = 0; i < n; ++i) mx = std::max(mx, fabs(x[i]));
  int e = 0;
  if (mx > 0.0) frexp(mx, &e);
  return e;
}

// Householder QR of the column-major m x n matrix W (overwritten):
// Q (m x r, orthonormal columns) and R (r x n), r = min(m, n), A = Q R.
inline void qr(int m, int n, double* W, double* Q, double* R, Work& wk) {
  const int r = std::min(m, n);
  // exact power-of-two prescaling: the squared norms below stay finite for
  // entries up to the top of the FP64 range (a long train's norm can reach
  // 2^800 before it is normalised)
  const int e = max_exponent((size_t)m * n, W);
  for (size_t i = 0; i < (size_t)m * n; ++i) W[i] = ldexp(W[i], -e);
  double* hv = grow(wk.hv, (size_t)m * r);  // Householder vector k in column k, rows k..m-1
  double* betas = grow(wk.betas, r);
  auto w = [&](int i, int j) -> double& { return W[(size_t)j * m + i]; };
  for (int k = 0; k < r; ++k) {
    double* v = hv + (size_t)k * m;
    double nrm = 0.0;
    for (int i = k; i < m; ++i) nrm += w(i, k) * w(i, k);
    nrm = sqrt(nrm);
    double beta = 0.0;
    for (int i = k; i < m; ++i) v[i] = 0.0;
    if (nrm > 0.0) {
      const double alpha = w(k, k) >= 0.0 ? -nrm : nrm;
      for (int i = k; i < m; ++i) v[i] = w(i, k);
      v[k] -= alpha;
      double vv = 0.0;
      for (int i = k; i < m; ++i) vv += v[i] * v[i];
      beta = vv > 0.0 ? 2.0 / vv : 0.0;
      for (int j = k; j < n; ++j) {
        double d = 0.0;
        for (int i = k; i < m; ++i) d += v[i] * w(i, j);
        d *= beta;
        for (int i = k; i < m; ++i) w(i, j) -= d * v[i];
      }
    }
    betas[k] = beta;
  }
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < r; ++i) R[(size_t)j * r + i] = i <= j ? ldexp(w(i, j), e) : 0.0;
  for (size_t i = 0; i < (size_t)m * r; ++i) Q[i] = 0.0;
  for (int j = 0; j < r; ++j) Q[(size_t)j * m + j] = 1.0;
  for (int k = r - 1; k >= 0; --k) {  // Q = H_0 ... H_{r-1} applied to the first r unit columns
    const double* v = hv + (size_t)k * m;
    for (int j = 0; j < r; ++j) {
      double* q = Q + (size_t)j * m;
      double d = 0.0;
      for (int i = k; i < m; ++i) d += v[i] * q[i];
      d *= betas[k];
      for (int i = k; i < m; ++i) q[i] -= d * v[i];
    }
  }
}

// Thin SVD A = U diag(S) V^T of the column-major m x n matrix A (m >= n) by
// one-sided Jacobi rotations (Hestenes); singular values decreasing.
// U is m x n, V is n x n, both column-major.
inline void svd_tall(int m, int n, const double* A, double* U, double* S, double* Vout, Work& wk) {
  double* W = grow(wk.W, (size_t)m * n);
  double* V = grow(wk.V, (size_t)n * n);
  double* nrm = grow(wk.nrm, n);
  const int e = max_exponent((size_t)m * n, A);  // exact prescaling, as in qr
  for (size_t i = 0; i < (size_t)m * n; ++i) W[i] = ldexp(A[i], -e);
  for (size_t i = 0; i < (size_t)n * n; ++i) V[i] = 0.0;
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 80; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double* wp = W + (size_t)p * m;
        double* wq = W + (size_t)q * m;
        double a = 0.0, b = 0.0, g = 0.0;
        for (int i = 0; i < m; ++i) {
          a += wp[i] * wp[i];
          b += wq[i] * wq[i];
          g += wp[i] * wq[i];
        }
        if (g == 0.0) continue;
        const double rel = fabs(g) / sqrt(a * b);
        off = std::max(off, rel);
        if (rel < 1e-15) continue;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < m; ++i) {
          const double x = wp[i], y = wq[i];
          wp[i] = c * x - s * y;
          wq[i] = s * x + c * y;
        }
        double* vp = V + (size_t)p * n;
        double* vq = V + (size_t)q * n;
        for (int i = 0; i < n; ++i) {
          const double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
      }
    if (off < 1e-15) break;
  }
  for (int j = 0; j < n; ++j) {
    double d = 0.0;
    for (int i = 0; i < m; ++i) d += W[(size_t)j * m + i] * W[(size_t)j * m + i];
    nrm[j] = sqrt(d);
  }
  wk.ord.resize(n);
  for (int j = 0; j < n; ++j) wk.ord[j] = j;
  std::sort(wk.ord.begin(), wk.ord.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
  for (int jj = 0; jj < n; ++jj) {
    const int j = wk.ord[jj];
    S[jj] = ldexp(nrm[j], e);
    for (int i = 0; i < m; ++i) U[(size_t)jj * m + i] = nrm[j] > 0.0 ? W[(size_t)j * m + i] / nrm[j] : 0.0;
    for (int i = 0; i < n; ++i) Vout[(size_t)jj * n + i] = V[(size_t)j * n + i];
  }
}

// thin SVD of any shape: U (m x r), S (r), V (n x r), r = min(m, n)
inline void svd(int m, int n, const double* A, double* U, double* S, double* V, Work& wk) {
  if (m >= n) { svd_tall(m, n, A, U, S, V, wk); return; }
  double* At = grow(wk.a, (size_t)m * n);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) At[(size_t)i * n + j] = A[(size_t)j * m + i];
  svd_tall(n, m, At, V, S, U, wk);  // A^T = V S U^T
}

inline void round_train(Train& t, int chi_max, double rel_tol) {
  const int L = t.L();
  Work& wk = work();
  // right-to-left: core k becomes right-orthonormal, R moves left
  for (int k = L - 1; k > 0; --k) {
    const int a = t.bond[k], b = t.bond[k + 1];
    const int m = 2 * b, r = std::min(m, a);
    double* Mt = grow(wk.b, (size_t)m * a);  // M^T, M[a][(s, b)], column-major m x a
    for (int s = 0; s < 2; ++s)
      for (int i = 0; i < a; ++i)
        for (int j = 0; j < b; ++j) Mt[(size_t)i * m + s * b + j] = t.at(k, s, i, j);
    double* Q = grow(wk.Q, (size_t)m * r);
    double* R = grow(wk.R, (size_t)r * a);
    qr(m, a, Mt, Q, R, wk);  // M = R^T Q^T
    std::vector<double>& cur = t.core[k];
    cur.assign((size_t)2 * r * b, 0.0);
    for (int s = 0; s < 2; ++s)
      for (int i = 0; i < r; ++i)
        for (int j = 0; j < b; ++j) cur[((size_t)s * r + i) * b + j] = Q[(size_t)i * m + s * b + j];
    const int x = t.bond[k - 1];
    double* pc = grow(wk.U, (size_t)2 * x * r);  // A_{k-1}[s] R^T
    for (int s = 0; s < 2; ++s)
      for (int i = 0; i < x; ++i)
        for (int j = 0; j < r; ++j) {
          double d = 0.0;
          for (int l = 0; l < a; ++l) d += t.at(k - 1, s, i, l) * R[(size_t)l * r + j];
          pc[((size_t)s * x + i) * r + j] = d;
        }
    t.core[k - 1].assign(pc, pc + (size_t)2 * x * r);
    t.bond[k] = r;
  }
  // left-to-right: truncated SVD, S V^T moves right
  for (int k = 0; k < L - 1; ++k) {
    const int a = t.bond[k], b = t.bond[k + 1];
    const int m = 2 * a, r = std::min(m, b);
    double* M = grow(wk.b, (size_t)m * b);  // M[(a, s)][b], column-major
    for (int s = 0; s < 2; ++s)
      for (int i = 0; i < a; ++i)
        for (int j = 0; j < b; ++j) M[(size_t)j * m + i * 2 + s] = t.at(k, s, i, j);
    double* U = grow(wk.U, (size_t)m * r);
    double* S = grow(wk.S, r);
    double* V = grow(wk.Vs, (size_t)b * r);
    svd(m, b, M, U, S, V, wk);
    int keep = 1;
    if (S[0] > 0.0) {
      keep = 0;
      for (int i = 0; i < r; ++i)
        if (S[i] > rel_tol * S[0]) ++keep;
      keep = std::max(1, std::min(chi_max, keep));
    }
    const int y = t.bond[k + 2];
    double* nx = grow(wk.R, (size_t)2 * keep * y);  // (S V^T) A_{k+1}[s]
    for (int s = 0; s < 2; ++s)
      for (int i = 0; i < keep; ++i)
        for (int j = 0; j < y; ++j) {
          double d = 0.0;
          for (int l = 0; l < b; ++l) d += S[i] * V[(size_t)i * b + l] * t.at(k + 1, s, l, j);
          nx[((size_t)s * keep + i) * y + j] = d;
        }
    std::vector<double>& cur = t.core[k];
    cur.assign((size_t)2 * a * keep, 0.0);
    for (int s = 0; s < 2; ++s)
      for (int i = 0; i < a; ++i)
        for (int j = 0; j < keep; ++j) cur[((size_t)s * a + i) * keep + j] = U[(size_t)j * m + i * 2 + s];
    t.core[k + 1].assign(nx, nx + (size_t)2 * keep * y);
    t.bond[k + 1] = keep;
  }
}

inline Train add(const Train& A, const Train& B) {
  const int L = A.L();
  Train C;
  C.bond.assign(L + 1, 0);
  C.core.resize(L);
  C.bond[0] = 1;
  C.bond[L] = 1;
  for (int k = 1; k < L; ++k) C.bond[k] = A.bond[k] + B.bond[k];
  if (L == 1) {
    C.core[0] = A.core[0];
    for (size_t i = 0; i < C.core[0].size(); ++i) C.core[0][i] += B.core[0][i];
    return C;
  }
  for (int k = 0; k < L; ++k) {
    const int a = C.bond[k], b = C.bond[k + 1];
    C.core[k].assign((size_t)2 * a * b, 0.0);
    const int ra = (k == 0) ? 0 : A.bond[k], cb = (k == L - 1) ? 0 : A.bond[k + 1];
    for (int s = 0; s < 2; ++s) {
      for (int i = 0; i < A.bond[k]; ++i)
        for (int j = 0; j < A.bond[k + 1]; ++j) C.core[k][((size_t)s * a + i) * b + j] = A.at(k, s, i, j);
      for (int i = 0; i < B.bond[k]; ++i)
        for (int j = 0; j < B.bond[k + 1]; ++j)
          C.core[k][((size_t)s * a + (ra + i)) * b + (cb + j)] = B.at(k, s, i, j);
    }
  }
  return C;
}

inline void scale(Train& t, double c) {
  for (double& x : t.core[0]) x *= c;
}

inline void apply_x(Train& t, const std::vector<int>& pi, int j) {
  for (int k = 0; k < t.L(); ++k)
    if (pi[k] == j) {
      const size_t h = t.core[k].size() / 2;
      std::swap_ranges(t.core[k].begin(), t.core[k].begin() + h, t.core[k].begin() + h);
    }
}

inline void apply_z(Train& t, const std::vector<int>& pi, int i) {
  for (int k = 0; k < t.L(); ++k)
    if (pi[k] == i) {
      const size_t h = t.core[k].size() / 2;
      for (size_t e = h; e < t.core[k].size(); ++e) t.core[k][e] = -t.core[k][e];
      return;
    }
}

// phi - tau H-bar phi for H-bar = J sum_bonds Zbar_i Zbar_j - h sum_j Xbar_j
// One Pauli string on the train: per position 0 = identity, 1 = X (slices
// swapped), 2 = Z (slice 1 negated), 3 = X Z (slice 1 negated, then swapped).
inline void apply_ops(Train& t, const uint8_t* ops) {
  for (int k = 0; k < t.L(); ++k) {
    if (ops[k] == 0) continue;
    const size_t n = t.core[k].size() / 2;
    double* c = t.core[k].data();
    if (ops[k] & 2)
      for (size_t e = 0; e < n; ++e) c[n + e] = -c[n + e];
    if (ops[k] & 1)
      for (size_t e = 0; e < n; ++e) std::swap(c[e], c[n + e]);
  }
}

// Sum of trains, two by two in order, each partial sum rounded.
// The sums of one level are independent: they run on up to 16 host threads.
inline Train pairwise_sum(std::vector<Train> terms, int chi_max, double rel_tol) {
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  while (terms.size() > 1) {
    const size_t pairs = terms.size() / 2;
    std::vector<Train> nxt((terms.size() + 1) / 2);
    std::atomic<bool> failed{false};
    auto work = [&](size_t p0, size_t p1) {
      try {
        for (size_t p = p0; p < p1; ++p) {
          nxt[p] = add(terms[2 * p], terms[2 * p + 1]);
          round_train(nxt[p], chi_max, rel_tol);
        }
      } catch (...) {  // an exception must not leave a worker thread
        failed = true;
      }
    };
    const size_t nt = std::min<size_t>(hw, pairs);
    if (nt <= 1) {
      work(0, pairs);
    } else {
      std::vector<std::thread> th;
      for (size_t w = 0; w < nt; ++w) th.emplace_back(work, pairs * w / nt, pairs * (w + 1) / nt);
      for (auto& t : th) t.join();
    }
    if (failed) throw std::bad_alloc();
    if (terms.size() % 2) nxt.back() = std::move(terms.back());
    terms.swap(nxt);
  }
  return std::move(terms[0]);
}

// alpha phi + beta sum_t c_t O_t phi: partial sums of the terms rounded to
// chi_sum, the result to chi_max.  With alpha = 1, beta = -tau and the
// strings of a replica-space Hamiltonian this is one power step; with
// alpha = 0, beta = 1 it applies an operator (a sum of strings) to phi.
inline Train pauli_apply(const Train& phi, int n_terms, const double* coeff, const uint8_t* ops, double alpha,
                         double beta, int chi_max, int chi_sum, double rel_tol) {
  std::vector<Train> terms;
  terms.reserve(n_terms);
  for (int t = 0; t < n_terms; ++t) {
    Train x = phi;
    apply_ops(x, ops + (size_t)t * phi.L());
    scale(x, coeff[t]);
    terms.push_back(std::move(x));
  }
  Train s = pairwise_sum(std::move(terms), chi_sum, rel_tol);
  scale(s, beta);
  if (alpha != 0.0) {
    Train a = phi;
    scale(a, alpha);
    s = add(a, s);
  }
  round_train(s, chi_max, rel_tol);
  return s;
}

// sum_m c_m phi_m: partial sums rounded to chi_max, the result once more.
inline Train combine(std::vector<Train> trains, const double* coeff, int chi_max, double rel_tol) {
  for (size_t m = 0; m < trains.size(); ++m) scale(trains[m], coeff[m]);
  Train s = pairwise_sum(std::move(trains), chi_max, rel_tol);
  round_train(s, chi_max, rel_tol);
  return s;
}

inline Train tfim_power_step(const Train& phi, const std::vector<int>& pi, int N,
                             const std::vector<std::pair<int, int>>& bonds, double J, double h, double tau,
                             int chi_max, double rel_tol) {
  std::vector<Train> terms;
  for (const auto& b : bonds) {
    Train t = phi;
    apply_z(t, pi, b.first);
    apply_z(t, pi, b.second);
    scale(t, J);
    terms.push_back(std::move(t));
  }
  for (int j = 0; j < N; ++j) {
    Train t = phi;
    apply_x(t, pi, j);
    scale(t, -h);
    terms.push_back(std::move(t));
  }
  Train hp = pairwise_sum(std::move(terms), chi_max, rel_tol);
  scale(hp, -tau);
  Train out = add(phi, hp);
  round_train(out, chi_max, rel_tol);
  return out;
}

}  // namespace rtt_tt
