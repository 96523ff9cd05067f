// Host-side operator construction for SFFT-based homogenization.
//
// These routines run once per grid size, reference medium or geometry
// (the paper's preprocessing, App. D) in FP64 on the host: small dense
// factorisations (Householder QR, one-sided Jacobi SVD) and TT-SVD.
#include "host_ops.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <stdexcept>

namespace qtt {
namespace host {

namespace {

inline double absq(double a) { return a * a; }
inline double absq(zc a) { return std::norm(a); }
inline double cj(double a) { return a; }
inline zc cj(zc a) { return std::conj(a); }
inline double re(double a) { return a; }
inline double re(zc a) { return a.real(); }

// Householder QR of a column-major m x n matrix A (lda = m).  On return
// Q (m x k, column-major) and R (k x n, column-major), k = min(m, n).
template <class T>
void house_qr(int m, int n, std::vector<T> A, std::vector<T>& Q, std::vector<T>& R) {
  const int k = std::min(m, n);
  std::vector<T> tau(k, T(0));
  for (int j = 0; j < k; ++j) {
    T* v = A.data() + (size_t)j * m;
    double xn2 = 0.0;
    for (int i = j + 1; i < m; ++i) xn2 += absq(v[i]);
    const T alpha = v[j];
    if (xn2 == 0.0 && std::abs(alpha - T(re(alpha))) == 0.0) { tau[j] = T(0); continue; }
    const double beta = -std::copysign(std::sqrt(absq(alpha) + xn2), re(alpha));
    tau[j] = (T(beta) - alpha) / T(beta);
    const T inv = T(1) / (alpha - T(beta));
    for (int i = j + 1; i < m; ++i) v[i] *= inv;
    v[j] = T(beta);
    for (int c = j + 1; c < n; ++c) {
      T* col = A.data() + (size_t)c * m;
      T s = col[j];
      for (int i = j + 1; i < m; ++i) s += cj(v[i]) * col[i];
      const T f = cj(tau[j]) * s;
      col[j] -= f;
      for (int i = j + 1; i < m; ++i) col[i] -= f * v[i];
    }
  }
  R.assign((size_t)k * n, T(0));
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= std::min(j, k - 1); ++i) R[i + (size_t)j * k] = A[i + (size_t)j * m];
  Q.assign((size_t)m * k, T(0));
  for (int j = 0; j < k; ++j) Q[j + (size_t)j * m] = T(1);
  for (int j = k - 1; j >= 0; --j) {
    if (tau[j] == T(0)) continue;
    const T* v = A.data() + (size_t)j * m;
    for (int c = j; c < k; ++c) {
      T* col = Q.data() + (size_t)c * m;
      T s = col[j];
      for (int i = j + 1; i < m; ++i) s += cj(v[i]) * col[i];
      const T f = tau[j] * s;
      col[j] -= f;
      for (int i = j + 1; i < m; ++i) col[i] -= f * v[i];
    }
  }
}

// One-sided Jacobi SVD, column-major m x n with m >= n.
template <class T>
void jacobi_svd(int m, int n, std::vector<T> A, std::vector<T>& U, std::vector<double>& S,
                std::vector<T>& V) {
  V.assign((size_t)n * n, T(0));
  for (int j = 0; j < n; ++j) V[j + (size_t)j * n] = T(1);
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rot = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        T* xa = A.data() + (size_t)p * m;
        T* xb = A.data() + (size_t)q * m;
        double al = 0, be = 0;
        T ga = T(0);
        for (int i = 0; i < m; ++i) {
          al += absq(xa[i]);
          be += absq(xb[i]);
          ga += cj(xa[i]) * xb[i];
        }
        const double g = std::abs(ga);
        if (!(g > tol * std::sqrt(al * be)) || al < 1e-300 || be < 1e-300) continue;
        rot = true;
        const double zeta = (be - al) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        const T ph = cj(ga) / T(g);
        for (int i = 0; i < m; ++i) {
          const T u = xa[i], w = ph * xb[i];
          xa[i] = c * u - s * w;
          xb[i] = s * u + c * w;
        }
        T* va = V.data() + (size_t)p * n;
        T* vb = V.data() + (size_t)q * n;
        for (int i = 0; i < n; ++i) {
          const T u = va[i], w = ph * vb[i];
          va[i] = c * u - s * w;
          vb[i] = s * u + c * w;
        }
      }
    if (!rot) break;
  }
  std::vector<double> sig(n);
  for (int j = 0; j < n; ++j) {
    double s2 = 0;
    for (int i = 0; i < m; ++i) s2 += absq(A[i + (size_t)j * m]);
    sig[j] = std::sqrt(s2);
  }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return sig[a] > sig[b]; });
  U.assign((size_t)m * n, T(0));
  std::vector<T> V2((size_t)n * n);
  S.resize(n);
  for (int jj = 0; jj < n; ++jj) {
    const int j = ord[jj];
    S[jj] = sig[j];
    for (int i = 0; i < m; ++i)
      U[i + (size_t)jj * m] = sig[j] > 0 ? A[i + (size_t)j * m] / T(sig[j]) : T(0);
    for (int i = 0; i < n; ++i) V2[i + (size_t)jj * n] = V[i + (size_t)j * n];
  }
  V.swap(V2);
}

// SVD of any column-major m x n matrix: A = Lft diag(S) Rgt^H with
// Lft (m x k), Rgt (n x k), k = min(m, n).
template <class T>
void svd_any(int m, int n, const std::vector<T>& A, std::vector<T>& Lft, std::vector<double>& S,
             std::vector<T>& Rgt) {
  if (m >= n) {
    std::vector<T> Q, R, U, V;
    if (m > 2 * n) {
      house_qr(m, n, A, Q, R);
      jacobi_svd(n, n, R, U, S, V);
      Lft.assign((size_t)m * n, T(0));
      for (int j = 0; j < n; ++j)
        for (int l = 0; l < n; ++l) {
          const T u = U[l + (size_t)j * n];
          if (u == T(0)) continue;
          for (int i = 0; i < m; ++i) Lft[i + (size_t)j * m] += Q[i + (size_t)l * m] * u;
        }
      Rgt = V;
    } else {
      jacobi_svd(m, n, A, Lft, S, Rgt);
    }
  } else {
    std::vector<T> Ah((size_t)n * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) Ah[j + (size_t)i * n] = cj(A[i + (size_t)j * m]);
    svd_any(n, m, Ah, Rgt, S, Lft);  // A^H = Rgt S Lft^H
  }
}

int keep_rank(const std::vector<double>& s, double thr, int cap) {
  const int k = (int)s.size();
  double tail = 0.0;
  int r = k;
  for (int i = k - 1; i >= 0; --i) {
    if (tail + s[i] * s[i] > thr * thr) break;
    tail += s[i] * s[i];
    r = i;
  }
  if (cap > 0) r = std::min(r, cap);
  return std::max(1, std::min(r, k));
}

int phys(const HCore& c) { return c.dout * std::max(c.din, 1); }

}  // namespace

HTT tt_svd_real(const std::vector<double>& T, const std::vector<int>& dims, double delta,
                int cap) {
  const int L = (int)dims.size();
  double nrm2 = 0;
  for (double v : T) nrm2 += v * v;
  const double thr = delta / std::sqrt(std::max(L - 1, 1)) * std::sqrt(nrm2);
  HTT out;
  // M is p x q row-major, stored as M^T column-major (q x p)
  std::vector<double> Mt = T;
  long q = (long)T.size();
  int r = 1;
  for (int k = 0; k < L - 1; ++k) {
    const int p = r * dims[k];
    q /= dims[k];
    // current buffer is row-major (r, dims[k], q) == row-major p x q == col-major q x p
    std::vector<double> Lm, Rm;
    std::vector<double> S;
    svd_any<double>((int)q, p, Mt, Lm, S, Rm);  // M^T = Lm S Rm^T  -> M = Rm S Lm^T
    const int rk = keep_rank(S, thr, cap);
    HCore c;
    c.r0 = r; c.dout = dims[k]; c.din = 0; c.r1 = rk;
    c.v.resize((size_t)p * rk);
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < rk; ++j) c.v[(size_t)i * rk + j] = Rm[i + (size_t)j * p];
    out.push_back(std::move(c));
    // next M = S Lm^T (rk x q) row-major == col-major q x rk = Lm * S
    std::vector<double> nx((size_t)q * rk);
    for (int j = 0; j < rk; ++j)
      for (long i = 0; i < q; ++i) nx[i + (size_t)j * q] = Lm[i + (size_t)j * q] * S[j];
    Mt.swap(nx);
    r = rk;
  }
  HCore last;
  last.r0 = r; last.dout = dims[L - 1]; last.din = 0; last.r1 = 1;
  last.v.resize((size_t)r * dims[L - 1]);
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < dims[L - 1]; ++j) last.v[(size_t)i * dims[L - 1] + j] = Mt[j + (size_t)i * dims[L - 1]];
  out.push_back(std::move(last));
  return out;
}

void tt_round(HTT& x, double delta, int cap) {
  const int L = (int)x.size();
  // right-to-left orthogonalisation: core k (r0 x P*r1) = Lk Qk
  for (int k = L - 1; k > 0; --k) {
    HCore& c = x[k];
    const int P = phys(c);
    const int m = c.r0, n = P * c.r1;
    // A = core as m x n (row-major) -> need LQ: A^H = Q R  (n x m, col-major = conj of row-major A)
    std::vector<zc> Ah((size_t)n * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) Ah[j + (size_t)i * n] = std::conj(c.v[(size_t)i * n + j]);
    std::vector<zc> Q, R;
    house_qr<zc>(n, m, Ah, Q, R);
    const int kk = std::min(m, n);
    // new core = Q^H (kk x n) row-major
    std::vector<zc> nv((size_t)kk * n);
    for (int i = 0; i < kk; ++i)
      for (int j = 0; j < n; ++j) nv[(size_t)i * n + j] = std::conj(Q[j + (size_t)i * n]);
    c.v.swap(nv);
    c.r0 = kk;
    // previous core *= R^H (m x kk): Rh[i][l] = conj(R[l][i]); R col-major kk x m
    HCore& pcore = x[k - 1];
    const int rows = pcore.r0 * phys(pcore);
    std::vector<zc> pv((size_t)rows * kk, zc(0));
    for (int a = 0; a < rows; ++a)
      for (int i = 0; i < m; ++i) {
        const zc v = pcore.v[(size_t)a * m + i];
        if (v == zc(0)) continue;
        for (int l = 0; l < kk; ++l) pv[(size_t)a * kk + l] += v * std::conj(R[l + (size_t)i * kk]);
      }
    pcore.v.swap(pv);
    pcore.r1 = kk;
  }
  double nrm2 = 0;
  for (const zc& v : x[0].v) nrm2 += std::norm(v);
  const double thr = delta / std::sqrt(std::max(L - 1, 1)) * std::sqrt(nrm2);
  for (int k = 0; k < L - 1; ++k) {
    HCore& c = x[k];
    const int p = c.r0 * phys(c), n = c.r1;
    std::vector<zc> A((size_t)p * n);
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < n; ++j) A[i + (size_t)j * p] = c.v[(size_t)i * n + j];
    std::vector<zc> Lf, Rg;
    std::vector<double> S;
    svd_any<zc>(p, n, A, Lf, S, Rg);
    const int rk = keep_rank(S, thr, cap);
    std::vector<zc> nv((size_t)p * rk);
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < rk; ++j) nv[(size_t)i * rk + j] = Lf[i + (size_t)j * p];
    c.v.swap(nv);
    c.r1 = rk;
    // next core = (S Rg^H)[:rk] * next  ; Rg is n x kmin col-major
    HCore& nc = x[k + 1];
    const int cols = phys(nc) * nc.r1;
    std::vector<zc> nn((size_t)rk * cols, zc(0));
    for (int a = 0; a < rk; ++a)
      for (int l = 0; l < n; ++l) {
        const zc w = S[a] * std::conj(Rg[l + (size_t)a * n]);
        if (w == zc(0)) continue;
        for (int j = 0; j < cols; ++j) nn[(size_t)a * cols + j] += w * nc.v[(size_t)l * cols + j];
      }
    nc.v.swap(nn);
    nc.r0 = rk;
  }
}

namespace {

// Operator product C = L * T core by core (apply T first, then L).
HTT op_times(const HTT& Lop, const HTT& Top) {
  HTT out(Lop.size());
  for (size_t k = 0; k < Lop.size(); ++k) {
    const HCore& a = Lop[k];
    const HCore& b = Top[k];
    HCore c;
    c.r0 = a.r0 * b.r0; c.r1 = a.r1 * b.r1; c.dout = a.dout; c.din = b.din;
    const int dm = a.din;  // == b.dout
    c.v.assign((size_t)c.r0 * c.dout * c.din * c.r1, zc(0));
    for (int ka = 0; ka < a.r0; ++ka)
      for (int kb = 0; kb < b.r0; ++kb)
        for (int o = 0; o < c.dout; ++o)
          for (int i = 0; i < c.din; ++i)
            for (int ka2 = 0; ka2 < a.r1; ++ka2)
              for (int kb2 = 0; kb2 < b.r1; ++kb2) {
                zc s = 0;
                for (int mm = 0; mm < dm; ++mm)
                  s += a.v[(((size_t)ka * a.dout + o) * a.din + mm) * a.r1 + ka2] *
                       b.v[(((size_t)kb * b.dout + mm) * b.din + i) * b.r1 + kb2];
                c.v[((((size_t)(ka * b.r0 + kb) * c.dout + o) * c.din + i) * c.r1) +
                    (ka2 * b.r1 + kb2)] = s;
              }
    out[k] = std::move(c);
  }
  return out;
}

HCore op_core(int r0, int r1) {
  HCore c;
  c.r0 = r0; c.r1 = r1; c.dout = 2; c.din = 2;
  c.v.assign((size_t)r0 * 4 * r1, zc(0));
  return c;
}
inline zc& at(HCore& c, int a, int o, int i, int b) {
  return c.v[(((size_t)a * c.dout + o) * c.din + i) * c.r1 + b];
}

}  // namespace

HTT qn_tto(int n, double delta) {
  const double PI = 3.14159265358979323846;
  const double h = 1.0 / std::sqrt(2.0);
  HTT T(n);
  for (int a = 0; a < n; ++a) {
    T[a] = op_core(1, 1);
    at(T[a], 0, 0, 0, 0) = 1.0;
    at(T[a], 0, 1, 1, 0) = 1.0;
  }
  // layer b: Hadamard on qubit b, then controlled phases pi/2^(a-b) between
  // the output bit of qubit b and the (still untouched) bit of qubit a > b.
  for (int b = 0; b < n; ++b) {
    HTT layer(n);
    for (int a = 0; a < n; ++a) {
      if (a < b) {
        layer[a] = op_core(1, 1);
        at(layer[a], 0, 0, 0, 0) = 1.0;
        at(layer[a], 0, 1, 1, 0) = 1.0;
      } else if (a == b) {
        const int r1 = (b == n - 1) ? 1 : 2;
        layer[a] = op_core(1, r1);
        for (int o = 0; o < 2; ++o)
          for (int i = 0; i < 2; ++i) {
            const double hv = (o == 1 && i == 1) ? -h : h;
            at(layer[a], 0, o, i, r1 == 1 ? 0 : o) = hv;
          }
      } else {
        const int r1 = (a == n - 1) ? 1 : 2;
        layer[a] = op_core(2, r1);
        for (int kap = 0; kap < 2; ++kap)
          for (int j = 0; j < 2; ++j) {
            const double th = PI * kap * j / std::ldexp(1.0, a - b);
            at(layer[a], kap, j, j, r1 == 1 ? 0 : kap) = std::polar(1.0, th);
          }
      }
    }
    T = op_times(layer, T);
    tt_round(T, 1e-15, 0);
  }
  tt_round(T, delta, 0);
  return T;
}

void iso_voigt(double lam, double mu, double C[36]) {
  for (int i = 0; i < 36; ++i) C[i] = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[i * 6 + j] = lam;
  for (int i = 0; i < 3; ++i) C[i * 6 + i] += 2.0 * mu;
  for (int i = 3; i < 6; ++i) C[i * 6 + i] = mu;
}

void iso_voigt_dim(int voigt, double lam, double mu, double* C) {
  if (voigt == 6) {
    iso_voigt(lam, mu, C);
    return;
  }
  // plane strain (11, 22, 12)
  const double v[9] = {lam + 2 * mu, lam, 0.0, lam, lam + 2 * mu, 0.0, 0.0, 0.0, mu};
  for (int i = 0; i < 9; ++i) C[i] = v[i];
}

namespace {

int bitrev(int k, int n) {
  int r = 0;
  for (int b = 0; b < n; ++b) r |= ((k >> b) & 1) << (n - 1 - b);
  return r;
}

// 1D momentum-order frequency tables: entry k holds the frequency of DFT
// index (-rev(k)) mod N (Nyquist represented as -N/2) and the same with the
// Nyquist sign flipped.
}  // namespace

void momentum_freqs(int n, std::vector<double>& f, std::vector<double>& f2) {
  const int N = 1 << n;
  f.resize(N);
  f2.resize(N);
  for (int k = 0; k < N; ++k) {
    const int m = (N - bitrev(k, n)) % N;
    const double fr = (m < N / 2) ? m : m - N;
    f[k] = fr;
    f2[k] = (m == N / 2) ? -fr : fr;
  }
}


HTT direction_train(int n, double delta) {
  const int N = 1 << n;
  std::vector<double> f, f2;
  momentum_freqs(n, f, f2);
  const size_t NN = (size_t)N * N * N;
  std::vector<double> T(6 * NN);
  for (int x = 0; x < N; ++x)
    for (int y = 0; y < N; ++y)
      for (int z = 0; z < N; ++z) {
        const size_t e = ((size_t)x * N + y) * N + z;
        const double r2 = f[x] * f[x] + f[y] * f[y] + f[z] * f[z];
        const double inv = r2 > 0 ? 1.0 / std::sqrt(r2) : 0.0;
        T[0 * NN + e] = f[x] * inv;
        T[1 * NN + e] = f[y] * inv;
        T[2 * NN + e] = f[z] * inv;
        T[3 * NN + e] = f2[x] * inv;
        T[4 * NN + e] = f2[y] * inv;
        T[5 * NN + e] = f2[z] * inv;
      }
  std::vector<int> dims(3 * n + 1, 2);
  dims[0] = 6;
  return tt_svd_real(T, dims, delta, 0);
}

namespace {

int voigt_index(int i, int j) {
  if (i == j) return i;
  const int a = std::min(i, j), b = std::max(i, j);
  if (a == 1 && b == 2) return 3;
  if (a == 0 && b == 2) return 4;
  return 5;  // (0, 1)
}

// operator whose control core is coef[out][in][c] contracted with the
// direction train's first core (c = (sigma, a)), spatial cores shared.
HTT control_op(const HTT& nt, int dout, int din, const std::vector<double>& coef, int nc = 6) {
  HTT op;
  HCore c0;
  const int r1 = nt[0].r1;
  c0.r0 = 1; c0.dout = dout; c0.din = din; c0.r1 = r1;
  c0.v.assign((size_t)dout * din * r1, zc(0));
  for (int o = 0; o < dout; ++o)
    for (int i = 0; i < din; ++i)
      for (int c = 0; c < nc; ++c) {
        const double w = coef[((size_t)o * din + i) * nc + c];
        if (w == 0.0) continue;
        for (int a = 0; a < r1; ++a)
          c0.v[((size_t)o * din + i) * r1 + a] += w * nt[0].v[(size_t)c * r1 + a];
      }
  op.push_back(std::move(c0));
  for (size_t k = 1; k < nt.size(); ++k) op.push_back(nt[k]);
  return op;
}

}  // namespace

GreenFactors green_factors(int n, double lam0, double mu0, double delta) {
  return green_factors_from(direction_train(n, delta), lam0, mu0);
}

GreenFactors green_factors_from(const HTT& nt, double lam0, double mu0) {
  GreenFactors G;
  // U: u^s_j = sum_k tau_{V(j,k)} n^s_k  ; out (s, j), in Voigt J
  {
    std::vector<double> cf(6 * 6 * 6, 0.0);
    for (int s = 0; s < 2; ++s)
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) cf[((size_t)(s * 3 + j) * 6 + voigt_index(j, k)) * 6 + s * 3 + k] += 1.0;
    G.U = control_op(nt, 6, 6, cf);
  }
  // Sd: s^s = sum_j u^s_j n^s_j ; out s (2), in (s, j)
  {
    std::vector<double> cf(2 * 6 * 6, 0.0);
    for (int s = 0; s < 2; ++s)
      for (int j = 0; j < 3; ++j) cf[((size_t)s * 6 + s * 3 + j) * 6 + s * 3 + j] = 1.0;
    G.Sd = control_op(nt, 2, 6, cf);
  }
  // P: p^s_j = n^s_j s^s ; out (s, j), in s
  {
    std::vector<double> cf(6 * 2 * 6, 0.0);
    for (int s = 0; s < 2; ++s)
      for (int j = 0; j < 3; ++j) cf[((size_t)(s * 3 + j) * 2 + s) * 6 + s * 3 + j] = 1.0;
    G.P = control_op(nt, 6, 2, cf);
  }
  // E: eps_V[I] = w_I * 1/2 sum_s (n^s_i q^s_j + n^s_j q^s_i), (i, j) = pair(I)
  {
    const int VP[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};
    const double W[6] = {1, 1, 1, 2, 2, 2};
    std::vector<double> cf(6 * 6 * 6, 0.0);
    for (int I = 0; I < 6; ++I) {
      const int i = VP[I][0], j = VP[I][1];
      for (int s = 0; s < 2; ++s) {
        // coefficient of q^s_j times n^s_i, and of q^s_i times n^s_j
        cf[((size_t)I * 6 + s * 3 + j) * 6 + s * 3 + i] += 0.5 * W[I];
        cf[((size_t)I * 6 + s * 3 + i) * 6 + s * 3 + j] += 0.5 * W[I];
      }
    }
    G.E = control_op(nt, 6, 6, cf);
  }
  green_scalars(lam0, mu0, &G.inv_2mu0, &G.half_c);
  return G;
}

void staggered_symbols(int n, std::vector<double>& kp, std::vector<double>& km) {
  const int N = 1 << n;
  kp.resize(2 * (size_t)N);
  km.resize(2 * (size_t)N);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < N; ++k) {
    const int m = (N - bitrev(k, n)) % N;
    const double h = pi * m / N;  // q / 2
    // exp(i q) - 1 = 2 i sin(q/2) exp(i q/2) = (-2 sin^2(q/2), sin q);
    // 1 - exp(-i q) = 2 i sin(q/2) exp(-i q/2) = (2 sin^2(q/2), sin q)
    const double s2 = 2.0 * std::sin(h) * std::sin(h), sq = std::sin(2.0 * h);
    kp[2 * k] = -s2;
    kp[2 * k + 1] = sq;
    km[2 * k] = s2;
    km[2 * k + 1] = sq;
  }
}

GreenFactors green_factors_staggered_from(const HTT& nt, double lam0, double mu0) {
  GreenFactors G;
  // control index c: a (0..2) -> n_a, 3 + a -> m_a
  // U: u_k = -m_k tau_kk - sum_{j != k} n_j tau_{V(k,j)} ; out k (3), in Voigt (6)
  {
    std::vector<double> cf(3 * 6 * 6, 0.0);
    for (int k = 0; k < 3; ++k) {
      cf[((size_t)k * 6 + k) * 6 + 3 + k] = -1.0;
      for (int j = 0; j < 3; ++j)
        if (j != k) cf[((size_t)k * 6 + voigt_index(k, j)) * 6 + j] = -1.0;
    }
    G.U = control_op(nt, 3, 6, cf);
  }
  // Sd: s = sum_k n_k u_k ; out 1, in 3
  {
    std::vector<double> cf(1 * 3 * 6, 0.0);
    for (int k = 0; k < 3; ++k) cf[(size_t)k * 6 + k] = 1.0;
    G.Sd = control_op(nt, 1, 3, cf);
  }
  // P: p_k = m_k s ; out 3, in 1
  {
    std::vector<double> cf(3 * 1 * 6, 0.0);
    for (int k = 0; k < 3; ++k) cf[(size_t)k * 6 + 3 + k] = 1.0;
    G.P = control_op(nt, 3, 1, cf);
  }
  // E: eps_kk = n_k q_k, gamma_ij = m_j q_i + m_i q_j ; out Voigt (6), in 3
  {
    const int VP[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};
    std::vector<double> cf(6 * 3 * 6, 0.0);
    for (int I = 0; I < 6; ++I) {
      const int i = VP[I][0], j = VP[I][1];
      if (i == j) {
        cf[((size_t)I * 3 + i) * 6 + i] = 1.0;
      } else {
        cf[((size_t)I * 3 + i) * 6 + 3 + j] += 1.0;
        cf[((size_t)I * 3 + j) * 6 + 3 + i] += 1.0;
      }
    }
    G.E = control_op(nt, 6, 3, cf);
  }
  green_scalars_scheme(1, lam0, mu0, &G.inv_2mu0, &G.half_c);
  return G;
}

GreenFactors green_factors_staggered2d_from(const HTT& nt, double lam0, double mu0) {
  GreenFactors G;
  // control c: a (0, 1) -> n_a, 2 + a -> m_a; plane Voigt (11, 22, 12)
  // U: u_k = -m_k tau_kk - n_j tau_12 (j != k) ; out 2, in 3
  {
    std::vector<double> cf(2 * 3 * 4, 0.0);
    for (int k = 0; k < 2; ++k) {
      cf[((size_t)k * 3 + k) * 4 + 2 + k] = -1.0;
      cf[((size_t)k * 3 + 2) * 4 + (1 - k)] = -1.0;
    }
    G.U = control_op(nt, 2, 3, cf, 4);
  }
  // Sd: s = sum_k n_k u_k ; out 1, in 2
  {
    std::vector<double> cf(1 * 2 * 4, 0.0);
    for (int k = 0; k < 2; ++k) cf[(size_t)k * 4 + k] = 1.0;
    G.Sd = control_op(nt, 1, 2, cf, 4);
  }
  // P: p_k = m_k s ; out 2, in 1
  {
    std::vector<double> cf(2 * 1 * 4, 0.0);
    for (int k = 0; k < 2; ++k) cf[(size_t)k * 4 + 2 + k] = 1.0;
    G.P = control_op(nt, 2, 1, cf, 4);
  }
  // E: eps_kk = n_k q_k, gamma_12 = m_2 q_1 + m_1 q_2 ; out 3, in 2
  {
    std::vector<double> cf(3 * 2 * 4, 0.0);
    for (int k = 0; k < 2; ++k) cf[((size_t)k * 2 + k) * 4 + k] = 1.0;
    cf[((size_t)2 * 2 + 0) * 4 + 2 + 1] += 1.0;
    cf[((size_t)2 * 2 + 1) * 4 + 2 + 0] += 1.0;
    G.E = control_op(nt, 3, 2, cf, 4);
  }
  green_scalars_scheme(1, lam0, mu0, &G.inv_2mu0, &G.half_c);
  return G;
}

GreenFactors green_factors2d_from(const HTT& nt, double lam0, double mu0) {
  GreenFactors G;
  // control c = 2 sigma + a (the two Nyquist representatives, axes x, y);
  // plane-strain Voigt (11, 22, 12)
  const int V2[2][2] = {{0, 2}, {2, 1}};
  // U: u^s_j = sum_k tau_{V(j,k)} n^s_k ; out (s, j) 4, in Voigt 3
  {
    std::vector<double> cf(4 * 3 * 4, 0.0);
    for (int s = 0; s < 2; ++s)
      for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 2; ++k) cf[((size_t)(s * 2 + j) * 3 + V2[j][k]) * 4 + s * 2 + k] += 1.0;
    G.U = control_op(nt, 4, 3, cf, 4);
  }
  // Sd: s^s = sum_j u^s_j n^s_j ; out s (2), in (s, j) 4
  {
    std::vector<double> cf(2 * 4 * 4, 0.0);
    for (int s = 0; s < 2; ++s)
      for (int j = 0; j < 2; ++j) cf[((size_t)s * 4 + s * 2 + j) * 4 + s * 2 + j] = 1.0;
    G.Sd = control_op(nt, 2, 4, cf, 4);
  }
  // P: p^s_j = n^s_j s^s ; out (s, j) 4, in s 2
  {
    std::vector<double> cf(4 * 2 * 4, 0.0);
    for (int s = 0; s < 2; ++s)
      for (int j = 0; j < 2; ++j) cf[((size_t)(s * 2 + j) * 2 + s) * 4 + s * 2 + j] = 1.0;
    G.P = control_op(nt, 4, 2, cf, 4);
  }
  // E: eps_I = w_I 1/2 sum_s (n^s_i q^s_j + n^s_j q^s_i), (i, j) = pair(I)
  {
    const int VP[3][2] = {{0, 0}, {1, 1}, {0, 1}};
    const double W[3] = {1, 1, 2};
    std::vector<double> cf(3 * 4 * 4, 0.0);
    for (int I = 0; I < 3; ++I) {
      const int i = VP[I][0], j = VP[I][1];
      for (int s = 0; s < 2; ++s) {
        cf[((size_t)I * 4 + s * 2 + j) * 4 + s * 2 + i] += 0.5 * W[I];
        cf[((size_t)I * 4 + s * 2 + i) * 4 + s * 2 + j] += 0.5 * W[I];
      }
    }
    G.E = control_op(nt, 3, 4, cf, 4);
  }
  green_scalars(lam0, mu0, &G.inv_2mu0, &G.half_c);
  return G;
}

void green_scalars_scheme(int scheme, double lam0, double mu0, double* a, double* c) {
  if (scheme == 0) {
    green_scalars(lam0, mu0, a, c);
    return;
  }
  *a = 1.0 / mu0;
  *c = -(lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0));
}

void green_scalars(double lam0, double mu0, double* inv_2mu0, double* half_c) {
  *inv_2mu0 = 0.5 / mu0;
  *half_c = 0.5 * (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0));
}

HTT stiffness_tto(const uint8_t* phase, int n, int nphase, const double* lame,
                  const double* lame0, double delta, int cap, HTT* chi, int* max_rank) {
  const size_t NN = (size_t)1 << (3 * n);
  std::vector<double> oh((size_t)nphase * NN, 0.0);
  for (size_t e = 0; e < NN; ++e) {
    const int p = phase[e];
    if (p >= nphase) throw std::invalid_argument("phase id out of range");
    oh[(size_t)p * NN + e] = 1.0;
  }
  std::vector<int> dims(3 * n + 1, 2);
  dims[0] = nphase;
  HTT t = tt_svd_real(oh, dims, delta, 0);
  return stiffness_from_chi(std::move(t), nphase, lame, lame0, cap, chi, max_rank, 6);
}

HTT stiffness_from_chi(HTT t, int nphase, const double* lame, const double* lame0, int cap, HTT* chi,
                       int* max_rank, int voigt) {
  int mr = 1;
  for (auto& c : t) mr = std::max(mr, c.r1);
  if (max_rank) *max_rank = mr;
  if (cap > 0 && mr > cap) throw std::length_error("stiffness rank exceeds cap");
  const int V = voigt, VV = V * V;
  double C0[36];
  iso_voigt_dim(V, lame0[0], lame0[1], C0);
  HTT op;
  HCore c0;
  const int r1 = t[0].r1;
  c0.r0 = 1; c0.dout = V; c0.din = V; c0.r1 = r1;
  c0.v.assign(VV * (size_t)r1, zc(0));
  for (int p = 0; p < nphase; ++p) {
    double Cp[36];
    iso_voigt_dim(V, lame[2 * p], lame[2 * p + 1], Cp);
    for (int I = 0; I < VV; ++I) {
      const double d = Cp[I] - C0[I];
      if (d == 0.0) continue;
      for (int a = 0; a < r1; ++a) c0.v[(size_t)I * r1 + a] += d * t[0].v[(size_t)p * r1 + a];
    }
  }
  op.push_back(std::move(c0));
  for (size_t k = 1; k < t.size(); ++k) op.push_back(t[k]);
  if (chi) *chi = std::move(t);
  return op;
}

}  // namespace host
}  // namespace qtt
