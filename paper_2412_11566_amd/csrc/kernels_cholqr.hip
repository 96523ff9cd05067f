// Orthonormal column bases by CholeskyQR2 on the FP64 matrix cores.
//
// The range finder of TT-rounding (Sec. 3) needs, per core, an orthonormal
// basis of the columns of a sketched unfolding (160 x 80 at rank cap 64),
// not its R factor.  CholeskyQR takes it from the Gram matrix:
// G = A^H A = R^H R (Cholesky), Q = A R^-1.  One pass leaves an
// orthogonality error of order u kappa(A)^2; a second pass on Q brings it to
// rounding level while u kappa(A)^2 stays well below one (CholeskyQR2:
// Yamamoto, Nakatsukasa, Yanagisawa and Fukaya, ETNA 2015).  Every step
// except the factorisation and inversion of the 16 x 16 diagonal blocks of
// R is a product of 16 x 16 blocks on v_mfma_f64_16x16x4f64, so one
// workgroup per matrix runs a chain of about fifteen barriers per pass
// instead of the two per column of an unblocked Householder QR.
//
// Second pass: when the Gram of the first pass's Q is within 1e-9 of the
// identity in Frobenius norm (E = G - I), R = I + U with U the upper
// triangle of E (diagonal halved) has R^H R = G - U^H U, and I - U inverts
// it to the same order (1e-18), so that pass needs no factorisation.
//
// Fallback: a first-pass Cholesky pivot that is not above 1e-12 of the
// largest diagonal entry (a rank-deficient A leaves pivots of rounding size,
// about n u of it, so it exits here, before the triangular solve), or a
// first-pass Q whose Gram is farther than 0.5 from the identity
// (Frobenius), flags the matrix; the Householder kernels
// then factor the flagged matrices later in the same stream, and skip the
// others.
//
// Lane layouts of v_mfma_f64_16x16x4f64 used below:
//   A: lane l holds A[l % 16][l / 16];  B: lane l holds B[l / 16][l % 16];
//   D: lane l, register r holds D[4 r + l / 16][l % 16].
// The triangular solve works on transposed blocks T_c = Q_c^T (16 columns
// of block c by the 16 rows of the wave's row block): in the D layout,
// register s of T_c is the B operand of the product's K-step s, so a lane
// reads back exactly the entries of the solved blocks it wrote itself.
#include "qtt_internal.h"
#include "fact_device.h"

#include <stdexcept>

namespace qtt {
namespace {

typedef double dv4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dv4 mf(double a, double b, dv4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// one K-step of a complex block product: (dr + i di) += (ar + i ai)(br + i bi)
__device__ __forceinline__ void cmf(double ar, double ai, double br, double bi, dv4& dr, dv4& di) {
  dr = mf(ar, br, dr);
  dr = mf(-ai, bi, dr);
  di = mf(ar, bi, di);
  di = mf(ai, br, di);
}

// orders LDS traffic between the lanes of one wave (no other wave takes part)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

constexpr int CQ_WAVES = 8;
constexpr int CQ_MAXM = 192;

// LDS layout in doubles: the Gram matrix, overwritten by the Cholesky
// factor, as real and imaginary planes of NP x (NP + 1); the inverses of the
// diagonal blocks as two planes of NB x 16 x 17.
template <int NB>
struct CqL {
  static constexpr int NP = 16 * NB, GS = NP + 1, BS = 16 * 17;
  static constexpr int GR = 0, GI = NP * GS, IR = 2 * NP * GS, II = IR + NB * BS;
  static constexpr int TOTAL = II + NB * BS;
};

// Broadcast of lane P of every 16-lane row to the whole row (DPP
// row_newbcast, control 0x150 + P): a register move, no LDS round trip.
template <int P>
__device__ __forceinline__ double bc(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x150 + P, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x150 + P, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One pivot of the diagonal-block Cholesky (rows below P updated, row P
// scaled into row P of R) and, in reverse order, one row of the inverse.
// Lane i (mod 16) holds row i; every 16-lane row of the wave holds the
// same copy, so row P reaches all lanes by bc<P>.  The block is Hermitian,
// so lane i already holds its multiplier G[i][P] = conj(G[P][i]).
template <int P>
struct CqStep {
  // the row masks enter as scalars (multiplier zero outside the rows that
  // change, scale one outside the pivot row), so a column costs its
  // broadcasts and fused multiply-adds and no selects
  static __device__ __forceinline__ void fact(cplx (&g)[16], double (&rd)[16], int i, double gmin, bool& bad) {
    const double d = bc<P>(g[P].x);
    const bool ok = d > gmin;  // false for NaN
    bad = bad || !ok;
    const double r = ok ? dev::rsq_nt(d) : 1.0;
    rd[P] = r;
    const double r2 = i > P ? r * r : 0.0;
    const cplx f = make_double2(g[P].x * r2, g[P].y * r2);  // G[i][P] / d below P, else 0
    const double sc = i == P ? r : 1.0;                      // row P becomes row P of R
#pragma unroll
    for (int j = P + 1; j < 16; ++j) {
      const cplx gpj = make_double2(bc<P>(g[j].x), bc<P>(g[j].y));
      cplx u = g[j];
      u.x = fma(-f.x, gpj.x, u.x);
      u.x = fma(f.y, gpj.y, u.x);
      u.y = fma(-f.x, gpj.y, u.y);
      u.y = fma(-f.y, gpj.x, u.y);
      g[j] = make_double2(u.x * sc, u.y * sc);
    }
    g[P] = dev::csel(i == P, make_double2(d * r, 0.0), g[P]);
    CqStep<P + 1>::fact(g, rd, i, gmin, bad);
  }
  // X[P] /= R[P][P]; X[i] -= R[i][P] X[P] for i < P; then row P - 1
  static __device__ __forceinline__ void inv(const cplx (&g)[16], const double (&rd)[16], cplx (&x)[16],
                                             int i) {
    const double sc = i == P ? rd[P] : 1.0;
    const cplx c = i < P ? g[P] : make_double2(0.0, 0.0);  // R[i][P] above P, else 0
#pragma unroll
    for (int j = P; j < 16; ++j) {
      x[j] = make_double2(x[j].x * sc, x[j].y * sc);
      const cplx xpj = make_double2(bc<P>(x[j].x), bc<P>(x[j].y));
      dev::caxpy_sub(x[j], c, xpj);
    }
    CqStep<P - 1>::inv(g, rd, x, i);
  }
};
template <>
struct CqStep<16> {
  static __device__ __forceinline__ void fact(cplx (&)[16], double (&)[16], int, double, bool&) {}
};
template <>
struct CqStep<-1> {
  static __device__ __forceinline__ void inv(const cplx (&)[16], const double (&)[16], cplx (&)[16], int) {}
};

// Cholesky factor and its inverse of diagonal block k (one wave): on entry
// the block in LDS holds the Schur complement (Hermitian, both triangles);
// on return it holds R_kk (upper, zero below) and Ir/Ii block k holds
// R_kk^-1.  Each of the 16 pivot steps is a handful of register
// broadcasts and fused multiply-adds, with no LDS round trip on the chain.
// A pivot not above gmin sets *fail.
template <int NB>
__device__ __forceinline__ void cq_diag(int k, double gmin, double* Gr, double* Gi, double* Ir, double* Ii,
                                        int lane, int* fail) {
  constexpr int GS = CqL<NB>::GS, BS = CqL<NB>::BS;
  const int i = lane & 15, o = 16 * k;
  cplx g[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int e = (o + i) * GS + o + j;
    g[j] = make_double2(Gr[e], Gi[e]);
  }
  bool bad = false;
  double rd[16];
  CqStep<0>::fact(g, rd, i, gmin, bad);
  if (bad && lane == 0) *fail = 1;
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int e = (o + i) * GS + o + j;
      Gr[e] = j < i ? 0.0 : g[j].x;
      Gi[e] = j < i ? 0.0 : g[j].y;
    }
  }
  cplx x[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) x[j] = make_double2(j == i ? 1.0 : 0.0, 0.0);
  CqStep<15>::inv(g, rd, x, i);
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int e = k * BS + i * 17 + j;
      Ir[e] = x[j].x;
      Ii[e] = x[j].y;
    }
  }
}

template <int NB>
__global__ __launch_bounds__(CQ_WAVES * 64) void k_cholqr2(int m, int n, MatView A, MatOut Q, int* flag) {
  using L = CqL<NB>;
  constexpr int NP = L::NP, GS = L::GS, BS = L::BS;
  constexpr int NT = NB * (NB + 1) / 2;
  extern __shared__ double sm[];
  double* Gr = sm + L::GR;
  double* Gi = sm + L::GI;
  double* Ir = sm + L::IR;
  double* Ii = sm + L::II;
  __shared__ int s_fail;
  __shared__ double s_red[CQ_WAVES];
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lc = lane & 15, lg = lane >> 4;
  const int mb = (m + 15) / 16;
  const MatView QV{Q.base, Q.rs, Q.cs, Q.sb, 0};
  cplx* Qb = Q.base + (long)b * Q.sb;
  if (tid == 0) s_fail = 0;

#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    const MatView S = pass == 0 ? A : QV;
    // ---- Gram G = S^H S: upper blocks (I <= J), one block per wave at a
    // time, three real products per K-step (Gauss); 8 K-steps of loads in
    // flight ahead of their products
    double e2 = 0.0;
    for (int t = w; t < NT; t += CQ_WAVES) {
      int I = 0, tt = t;
      while (tt >= NB - I) {
        tt -= NB - I;
        ++I;
      }
      const int J = I + tt;
      const int cI = 16 * I + lc, cJ = 16 * J + lc;
      const bool okI = cI < n, okJ = cJ < n;
      dv4 p1 = {0.0, 0.0, 0.0, 0.0}, p2 = p1, p3 = p1;
      for (int k0 = 0; k0 < m; k0 += 32) {
        cplx va[8], vc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int row = k0 + 4 * u + lg;
          const bool okr = row < m;
          va[u] = (okr && okI) ? dev::ldv(S, b, row, cI) : make_double2(0.0, 0.0);
          vc[u] = (okr && okJ && I != J) ? dev::ldv(S, b, row, cJ) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const cplx a = va[u];
          const cplx c = dev::csel(I == J, va[u], vc[u]);
          // A = S^H: (a.x, -a.y); B = S: (c.x, c.y)
          p1 = mf(a.x, c.x, p1);
          p2 = mf(-a.y, c.y, p2);
          p3 = mf(a.x - a.y, c.x + c.y, p3);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = 16 * I + 4 * r + lg, gj = 16 * J + lc;
        double vr = p1[r] - p2[r], vi = p3[r] - p1[r] - p2[r];
        if (gi >= n || gj >= n) {
          vr = gi == gj ? 1.0 : 0.0;
          vi = 0.0;
        }
        Gr[gi * GS + gj] = vr;
        Gi[gi * GS + gj] = vi;
        const double dr = vr - (gi == gj ? 1.0 : 0.0);
        e2 += (I == J ? 1.0 : 2.0) * (dr * dr + vi * vi);
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) e2 += __shfl_xor(e2, o);
    if (lane == 0) s_red[w] = e2;
    __syncthreads();
    bool first_order = false;
    if (pass == 1) {
      double E2 = 0.0;
#pragma unroll
      for (int i = 0; i < CQ_WAVES; ++i) E2 += s_red[i];
      if (!(E2 <= 0.25)) {
        if (tid == 0) flag[b] = 1;
        return;
      }
      first_order = E2 <= 1e-18;
    }
    if (first_order) {
      // R = I + U: its off-diagonal blocks are those of G; diagonal-block
      // inverses I - U_cc
      for (int c = w; c < NB; c += CQ_WAVES) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = lg + 4 * q, j = lc, e = (16 * c + i) * GS + 16 * c + j;
          double vr = 0.0, vi = 0.0;
          if (i == j) {
            vr = 1.0 - 0.5 * (Gr[e] - 1.0);
          } else if (i < j) {
            vr = -Gr[e];
            vi = -Gi[e];
          }
          Ir[c * BS + i * 17 + j] = vr;
          Ii[c * BS + i * 17 + j] = vi;
        }
      }
      __syncthreads();
    } else {
      // blocked right-looking Cholesky, G = R^H R
      double gmin = 0.0;
      if (w == 0) {
        double gmax = 0.0;
        for (int j = lane; j < NP; j += 64) gmax = fmax(gmax, Gr[j * GS + j]);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, o));
        gmin = 1e-12 * gmax;
      }
      for (int k = 0; k < NB; ++k) {
        if (w == 0) cq_diag<NB>(k, gmin, Gr, Gi, Ir, Ii, lane, &s_fail);
        __syncthreads();
        if (s_fail) {
          if (tid == 0) flag[b] = 1;
          return;
        }
        // row panel R_kj = R_kk^-H G_kj, one block per wave
        for (int j = k + 1 + w; j < NB; j += CQ_WAVES) {
          dv4 dr = {0.0, 0.0, 0.0, 0.0}, di = dr;
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int kk = 4 * s4 + lg, e = (16 * k + kk) * GS + 16 * j + lc;
            const int ei = k * BS + kk * 17 + lc;
            cmf(Ir[ei], -Ii[ei], Gr[e], Gi[e], dr, di);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = (16 * k + 4 * r + lg) * GS + 16 * j + lc;
            Gr[e] = dr[r];
            Gi[e] = di[r];
          }
        }
        __syncthreads();
        // trailing update G_ij -= R_ki^H R_kj, k < i <= j
        const int nt = NB - k - 1, cnt = nt * (nt + 1) / 2;
        for (int t = w; t < cnt; t += CQ_WAVES) {
          int i = 0, tt = t;
          while (tt >= nt - i) {
            tt -= nt - i;
            ++i;
          }
          const int bi = k + 1 + i, bj = bi + tt;
          dv4 dr, di;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = (16 * bi + 4 * r + lg) * GS + 16 * bj + lc;
            dr[r] = Gr[e];
            di[r] = Gi[e];
          }
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int kr = (16 * k + 4 * s4 + lg) * GS;
            const int ea = kr + 16 * bi + lc, eb = kr + 16 * bj + lc;
            cmf(-Gr[ea], Gi[ea], Gr[eb], Gi[eb], dr, di);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = (16 * bi + 4 * r + lg) * GS + 16 * bj + lc;
            Gr[e] = dr[r];
            Gi[e] = di[r];
          }
        }
        __syncthreads();
      }
    }
    // ---- Q = S R^-1 by block forward substitution over column blocks, on
    // transposed blocks: T_c = R_cc^-T (S_c^T - sum_{c' < c} R_c'c^T T_c')
    for (int ib = w; ib < mb; ib += CQ_WAVES) {
      const int row = 16 * ib + lc;
      const bool okrow = row < m;
      cplx* qrow = Qb + (long)row * Q.rs;
#pragma unroll 1
      for (int c = 0; c < NB; ++c) {
        dv4 sr, si;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = 16 * c + 4 * r + lg;
          const cplx v = (okrow && col < n) ? dev::ldv(S, b, row, col) : make_double2(0.0, 0.0);
          sr[r] = v.x;
          si[r] = v.y;
        }
        // solved blocks T_c' come back from Q (this lane wrote them); the
        // products R_c'c^T T_c' accumulate as three real products (Gauss)
        dv4 p1 = {0.0, 0.0, 0.0, 0.0}, p2 = p1, p3 = p1;
#pragma unroll 1
        for (int c2 = 0; c2 < c; ++c2) {
          cplx t[4];
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int col = 16 * c2 + 4 * s4 + lg;
            t[s4] = (okrow && col < n) ? qrow[(long)col * Q.cs] : make_double2(0.0, 0.0);
          }
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int e = (16 * c2 + 4 * s4 + lg) * GS + 16 * c + lc;
            const double ar = Gr[e], ai = Gi[e];
            p1 = mf(ar, t[s4].x, p1);
            p2 = mf(ai, t[s4].y, p2);
            p3 = mf(ar + ai, t[s4].x + t[s4].y, p3);
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          sr[r] -= p1[r] - p2[r];
          si[r] -= p3[r] - p1[r] - p2[r];
        }
        dv4 q1 = {0.0, 0.0, 0.0, 0.0}, q2 = q1, q3 = q1;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int e = c * BS + (4 * s4 + lg) * 17 + lc;
          const double ar = Ir[e], ai = Ii[e];
          q1 = mf(ar, sr[s4], q1);
          q2 = mf(ai, si[s4], q2);
          q3 = mf(ar + ai, sr[s4] + si[s4], q3);
        }
        dv4 nr, ni;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          nr[r] = q1[r] - q2[r];
          ni[r] = q3[r] - q1[r] - q2[r];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = 16 * c + 4 * r + lg;
          if (okrow && col < n) qrow[(long)col * Q.cs] = make_double2(nr[r], ni[r]);
        }
      }
    }
    // the next pass reads Q written by every wave
    __syncthreads();
  }
  if (tid == 0) flag[b] = 0;
}

template <int NB>
void launch_cq(int batch, int m, int n, const MatView& A, const MatOut& Q, int* flag, hipStream_t s) {
  const size_t shm = (size_t)CqL<NB>::TOTAL * sizeof(double);
  // once per kernel and process (thread-safe static initialisation)
  static const bool attr = [&]() {
    check(hipFuncSetAttribute((const void*)k_cholqr2<NB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shm),
          "cholqr2 lds attribute");
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL((k_cholqr2<NB>), dim3(batch), dim3(CQ_WAVES * 64), shm, s, m, n, A, Q, flag);
  check(hipGetLastError(), "cholqr2 launch");
}

}  // namespace

// shapes the fallback's register kernel holds too: up to 192 rows, 168
// beyond 64 columns
bool orth_ok(int m, int n) { return m >= n && n > 16 && n <= 80 && m > 32 && m <= (n > 64 ? 168 : CQ_MAXM); }

size_t orth_ws(int batch, int m, int n) {
  return (size_t)(batch + 3) / 4 + (size_t)batch * n * n + qr_ws(batch, m, n);
}

bool orth(int batch, int m, int n, MatView A, MatOut Q, cplx* ws, hipStream_t s) {
  if (batch <= 0) return true;
  if (!orth_ok(m, n)) return false;
  int* flag = (int*)ws;
  cplx* Rs = ws + (batch + 3) / 4;
  cplx* hws = Rs + (size_t)batch * n * n;
  switch ((n + 15) / 16) {
    case 2: launch_cq<2>(batch, m, n, A, Q, flag, s); break;
    case 3: launch_cq<3>(batch, m, n, A, Q, flag, s); break;
    case 4: launch_cq<4>(batch, m, n, A, Q, flag, s); break;
    default: launch_cq<5>(batch, m, n, A, Q, flag, s); break;
  }
  // Householder for the flagged matrices (the others exit at once)
  const MatOut R{Rs, (long)n, 1, (long)n * n};
  if (!qr_2d_vectors(batch, m, n, A, R, hws, s, flag) || !qr_form_q(batch, m, n, Q, hws, s, flag))
    throw std::logic_error("orth: no Householder variant for the shape");
  return true;
}

}  // namespace qtt
