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
// diagonal blocks as two planes of NB x 16 x 17; two buffers of 16 complex
// values for the diagonal-block steps.
template <int NB>
struct CqL {
  static constexpr int NP = 16 * NB, GS = NP + 1, BS = 16 * 17;
  static constexpr int GR = 0, GI = NP * GS, IR = 2 * NP * GS, II = IR + NB * BS, MC = II + NB * BS;
  static constexpr int TOTAL = MC + 64;
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

// scalar broadcast of lane `src`'s value (src uniform across the wave)
__device__ __forceinline__ double rl(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One pivot of the diagonal-block Cholesky.  Lane (g, i) = 16 g + i holds
// row i at the columns g + 4 t, t < 4 (a[t]), so every lane does a quarter
// of a row.  The pivot comes from lane (P % 4, P) as a scalar (readlane);
// row P reaches the lanes of each 16-lane row by a DPP row broadcast from
// its lane P, which holds exactly that row's columns; the multipliers G[i][P]
// (column P, held by the lanes of group P % 4) reach every group by a lane
// permute.  All rows and columns beyond P are updated (both triangles:
// the lower one holds the multipliers of the later steps); row P becomes row
// P of R.
template <int P>
struct CqStep {
  static __device__ __forceinline__ void fact(cplx (&a)[4], double (&rd)[16], int g, int i, double gmin,
                                              bool drop, bool& bad, double* mc) {
    constexpr int gp = P & 3, tp = P >> 2;
    const double d = rl(a[tp].x, 16 * gp + P);
    const bool ok = d > gmin;  // false for NaN
    // a pivot at rounding level either fails the factorisation or, when
    // dropping, gives a zero row of R and a zero row and column of R^-1
    bad = bad || (drop ? d != d : !ok);
    const double r = ok ? dev::rsq_nt(d) : (drop ? 0.0 : 1.0);
    rd[P] = r;
    (void)mc;
    // G[i][P] from lane (P % 4, i) by a lane permute (no LDS round trip)
    const double gx = __shfl(a[tp].x, 16 * gp + i, 64), gy = __shfl(a[tp].y, 16 * gp + i, 64);
    const double r2 = i > P ? r * r : 0.0;
    const cplx f = make_double2(gx * r2, gy * r2);  // G[i][P] / d below P, else 0
    const double sc = i == P ? r : 1.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = g + 4 * t;
      const cplx gpj = make_double2(bc<P>(a[t].x), bc<P>(a[t].y));  // G[P][j]
      cplx u = a[t];
      u.x = fma(-f.x, gpj.x, u.x);
      u.x = fma(f.y, gpj.y, u.x);
      u.y = fma(-f.x, gpj.y, u.y);
      u.y = fma(-f.y, gpj.x, u.y);
      const cplx upd = make_double2(u.x * sc, u.y * sc);
      const cplx piv = dev::csel(i == P, make_double2(d * r, 0.0), a[t]);
      a[t] = dev::csel(j > P, upd, dev::csel(j == P, piv, a[t]));
    }
    CqStep<P + 1>::fact(a, rd, g, i, gmin, drop, bad, mc);
  }
  // X[P] /= R[P][P]; X[i] -= R[i][P] X[P] for i < P; then row P - 1.  Lane
  // (g, i) holds row i of X at the columns g + 4 t; R[i][P] comes from LDS.
  static __device__ __forceinline__ void inv(const double (&rd)[16], cplx (&x)[4], int i, const double* Rr,
                                             const double* Ri, int gs) {
    const double sc = i == P ? rd[P] : 1.0;
    const int e = i * gs + P;
    const cplx c = i < P ? make_double2(Rr[e], Ri[e]) : make_double2(0.0, 0.0);  // R[i][P] above P
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      x[t] = make_double2(x[t].x * sc, x[t].y * sc);
      const cplx xpj = make_double2(bc<P>(x[t].x), bc<P>(x[t].y));
      dev::caxpy_sub(x[t], c, xpj);
    }
    CqStep<P - 1>::inv(rd, x, i, Rr, Ri, gs);
  }
};
template <>
struct CqStep<16> {
  static __device__ __forceinline__ void fact(cplx (&)[4], double (&)[16], int, int, double, bool, bool&,
                                              double*) {}
};
template <>
struct CqStep<-1> {
  static __device__ __forceinline__ void inv(const double (&)[16], cplx (&)[4], int, const double*,
                                             const double*, int) {}
};

// Cholesky factor and its inverse of diagonal block k (one wave): on entry
// the block in LDS holds the Schur complement (Hermitian, both triangles);
// on return it holds R_kk (upper, zero below) and Ir/Ii block k holds
// R_kk^-1.  A pivot not above gmin sets *fail (unless dropping).
template <int NB>
__device__ __forceinline__ void cq_diag(int k, double gmin, bool drop, double* Gr, double* Gi, double* Ir,
                                        double* Ii, double* mc, int lane, int* fail) {
  constexpr int GS = CqL<NB>::GS, BS = CqL<NB>::BS;
  const int i = lane & 15, g = lane >> 4, o = 16 * k;
  cplx a[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int e = (o + i) * GS + o + g + 4 * t;
    a[t] = make_double2(Gr[e], Gi[e]);
  }
  bool bad = false;
  double rd[16];
  CqStep<0>::fact(a, rd, g, i, gmin, drop, bad, mc);
  if (bad && lane == 0) *fail = 1;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = g + 4 * t, e = (o + i) * GS + o + j;
    Gr[e] = j < i ? 0.0 : a[t].x;
    Gi[e] = j < i ? 0.0 : a[t].y;
  }
  wave_sync();
  cplx x[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) x[t] = make_double2(g + 4 * t == i ? 1.0 : 0.0, 0.0);
  CqStep<15>::inv(rd, x, i, Gr + o * GS + o, Gi + o * GS + o, GS);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int e = k * BS + i * 17 + g + 4 * t;
    Ir[e] = x[t].x;
    Ii[e] = x[t].y;
  }
}

// Second pass without factorisation (the Gram G of the first pass's Q is
// within 1e-9 of I): R = I + U, U the upper triangle of E = G - I with the
// diagonal halved; its off-diagonal blocks are those of G already, the
// diagonal-block inverses become I - U_cc.  Ends with a barrier.
template <int NB>
__device__ __forceinline__ void cq_first_order(double* Gr, double* Gi, double* Ir, double* Ii, int w, int lane) {
  constexpr int GS = CqL<NB>::GS, BS = CqL<NB>::BS;
  const int lc = lane & 15, lg = lane >> 4;
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
}

// Blocked right-looking Cholesky G = R^H R of the Gram in LDS by all waves
// of the workgroup: R overwrites the upper blocks of G, the inverses of the
// diagonal blocks go to Ir/Ii.  Returns false (uniformly) when a pivot is
// not above 1e-12 of the largest diagonal entry; with drop, pivots not above
// 1e-13 of it (a column dependent on the earlier ones to rounding) give a
// zero row of R and a zero row and column of R^-1 instead, so that column
// of Q = A R^-1 is exactly zero.  Ends with a barrier.
template <int NB>
__device__ __forceinline__ bool cq_cholesky(double* Gr, double* Gi, double* Ir, double* Ii, int w, int lane,
                                            bool drop, int* s_fail) {
  constexpr int NP = CqL<NB>::NP, GS = CqL<NB>::GS, BS = CqL<NB>::BS;
  const int lc = lane & 15, lg = lane >> 4;
  double gmin = 0.0;
  if (w == 0) {
    double gmax = 0.0;
    for (int j = lane; j < NP; j += 64) gmax = fmax(gmax, Gr[j * GS + j]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, o));
    gmin = (drop ? 1e-13 : 1e-12) * gmax;
  }
  for (int k = 0; k < NB; ++k) {
    if (w == 0) cq_diag<NB>(k, gmin, drop, Gr, Gi, Ir, Ii, Ir + (CqL<NB>::MC - CqL<NB>::IR), lane, s_fail);
    __syncthreads();
    if (*s_fail) return false;
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
  return true;
}

template <int NB>
__global__ __launch_bounds__(CQ_WAVES * 64) void k_cholqr2(int m, int n, MatView A, MatOut Q, int* flag, int drop) {
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
        // padding, and (second pass, dropping) the exactly zero columns of
        // dependent directions, enter as identity
        if (gi >= n || gj >= n || (drop && pass == 1 && gi == gj && vr == 0.0)) {
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
      cq_first_order<NB>(Gr, Gi, Ir, Ii, w, lane);
    } else if (!cq_cholesky<NB>(Gr, Gi, Ir, Ii, w, lane, drop != 0, &s_fail)) {
      if (tid == 0) flag[b] = 1;
      return;
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

// ---------------------------------------------------------------------------
// The same CholeskyQR2 spread over the device: each pass is a partial Gram
// per 32-row slice (one workgroup each), one workgroup per matrix that sums
// the slices, factors and inverts (R^-1 upper, by block back substitution),
// and the product S R^-1 on the library's batched GEMM.  The dependent chain
// of one compute unit shrinks to the Cholesky and the inverse.
// ---------------------------------------------------------------------------
constexpr int GP_ROWS = 32;  // matrix rows per partial Gram (8 K-steps)

// partial Gram blocks (I <= J) of rows [32 part, 32 part + 32) of matrix b:
// Gp[((b nparts + part) NT + t) 256 + 16 r + c], row-major 16 x 16 blocks
// one wave per block pair (NT <= 15 of the 16 waves): a single round of
// loads and products
template <int NB>
__global__ __launch_bounds__(1024) void k_gram_part(int m, int n, MatView S, cplx* Gp, int nparts) {
  constexpr int NT = NB * (NB + 1) / 2;
  const int part = blockIdx.x, b = blockIdx.y, lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lc = lane & 15, lg = lane >> 4;
  const int r0 = part * GP_ROWS, r1 = min(m, r0 + GP_ROWS);
  cplx* out = Gp + ((long)b * nparts + part) * NT * 256;
  for (int t = w; t < NT; t += 16) {
    int I = 0, tt = t;
    while (tt >= NB - I) {
      tt -= NB - I;
      ++I;
    }
    const int J = I + tt;
    const int cI = 16 * I + lc, cJ = 16 * J + lc;
    const bool okI = cI < n, okJ = cJ < n;
    cplx va[8], vc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int row = r0 + 4 * u + lg;
      const bool okr = row < r1;
      va[u] = (okr && okI) ? dev::ldv(S, b, row, cI) : make_double2(0.0, 0.0);
      vc[u] = (okr && okJ && I != J) ? dev::ldv(S, b, row, cJ) : make_double2(0.0, 0.0);
    }
    dv4 p1 = {0.0, 0.0, 0.0, 0.0}, p2 = p1, p3 = p1;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const cplx a = va[u];
      const cplx c = dev::csel(I == J, va[u], vc[u]);
      p1 = mf(a.x, c.x, p1);
      p2 = mf(-a.y, c.y, p2);
      p3 = mf(a.x - a.y, c.x + c.y, p3);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
      out[t * 256 + (4 * r + lg) * 16 + lc] = make_double2(p1[r] - p2[r], p3[r] - p1[r] - p2[r]);
  }
}

// Sum of the partial Grams (in slice order), then as in the fused kernel:
// pass 0 factors (or flags the matrix), pass 1 checks ||G - I||_F <= 0.5 and
// factors without a Cholesky when G is within 1e-9 of I.  Writes the full
// upper-triangular X = R^-1 (n x n, zero below) for the product S X.  A
// matrix flagged by pass 0 is skipped by pass 1.
template <int NB>
__global__ __launch_bounds__(CQ_WAVES * 64) void k_chol_inv(int n, const cplx* Gp, int nparts, cplx* X,
                                                            int* flag, int pass, int drop) {
  using L = CqL<NB>;
  constexpr int GS = L::GS, BS = L::BS, NT = NB * (NB + 1) / 2;
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
  if (pass == 1 && flag[b] != 0) return;
  if (tid == 0) s_fail = 0;
  // the partial Grams summed in slice order; each thread's EPT elements are
  // loaded together per slice (two slices per round), so the dependent
  // chain is one load round trip per two slices, not one per element and
  // slice
  constexpr int NE = NT * 256, EPT = (NE + CQ_WAVES * 64 - 1) / (CQ_WAVES * 64);
  double ar[EPT], ai[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) ar[u] = ai[u] = 0.0;
  {
    const cplx* gb = Gp + (long)b * nparts * NE;
    int p = 0;
    for (; p + 2 <= nparts; p += 2) {
      cplx v0[EPT], v1[EPT];
#pragma unroll
      for (int u = 0; u < EPT; ++u) {
        const int e = tid + u * CQ_WAVES * 64;
        v0[u] = e < NE ? gb[(long)p * NE + e] : make_double2(0.0, 0.0);
        v1[u] = e < NE ? gb[(long)(p + 1) * NE + e] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < EPT; ++u) {
        ar[u] += v0[u].x;
        ai[u] += v0[u].y;
        ar[u] += v1[u].x;
        ai[u] += v1[u].y;
      }
    }
    if (p < nparts) {
#pragma unroll
      for (int u = 0; u < EPT; ++u) {
        const int e = tid + u * CQ_WAVES * 64;
        const cplx v = e < NE ? gb[(long)p * NE + e] : make_double2(0.0, 0.0);
        ar[u] += v.x;
        ai[u] += v.y;
      }
    }
  }
  double e2 = 0.0;
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = tid + u * CQ_WAVES * 64;
    if (e >= NE) break;
    const int t = e >> 8, q = e & 255;
    int I = 0, tt = t;
    while (tt >= NB - I) {
      tt -= NB - I;
      ++I;
    }
    const int J = I + tt;
    double vr = ar[u], vi = ai[u];
    const int gi = 16 * I + (q >> 4), gj = 16 * J + (q & 15);
    if (gi >= n || gj >= n || (drop && pass == 1 && gi == gj && vr == 0.0)) {
      vr = gi == gj ? 1.0 : 0.0;
      vi = 0.0;
    }
    Gr[gi * GS + gj] = vr;
    Gi[gi * GS + gj] = vi;
    const double dr = vr - (gi == gj ? 1.0 : 0.0);
    e2 += (I == J ? 1.0 : 2.0) * (dr * dr + vi * vi);
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
    cq_first_order<NB>(Gr, Gi, Ir, Ii, w, lane);
  } else {
    if (!cq_cholesky<NB>(Gr, Gi, Ir, Ii, w, lane, drop != 0, &s_fail)) {
      if (tid == 0) flag[b] = 1;
      return;
    }
    // X_ij = -R_ii^-1 sum_{i < l <= j} R_il X_lj by diagonals d = j - i, one
    // block per wave; X_ij (i < j) is kept in the unused lower block (j, i)
    // of the LDS matrix, element (r, c) at row 16 j + r, column 16 i + c
    for (int d = 1; d < NB; ++d) {
      for (int i = w; i + d < NB; i += CQ_WAVES) {
        const int j = i + d;
        dv4 t1 = {0.0, 0.0, 0.0, 0.0}, t2 = t1, t3 = t1;
        for (int l = i + 1; l <= j; ++l) {
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int ea = (16 * i + lc) * GS + 16 * l + 4 * s4 + lg;  // R_il[lc][4 s4 + lg]
            double br, bi;
            if (l == j) {
              const int ex = j * BS + (4 * s4 + lg) * 17 + lc;
              br = Ir[ex];
              bi = Ii[ex];
            } else {
              const int ex = (16 * j + 4 * s4 + lg) * GS + 16 * l + lc;
              br = Gr[ex];
              bi = Gi[ex];
            }
            const double ar = Gr[ea], ai = Gi[ea];
            t1 = mf(ar, br, t1);
            t2 = mf(ai, bi, t2);
            t3 = mf(ar + ai, br + bi, t3);
          }
        }
        dv4 tr, ti;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          tr[r] = t1[r] - t2[r];
          ti[r] = t3[r] - t1[r] - t2[r];
        }
        dv4 u1 = {0.0, 0.0, 0.0, 0.0}, u2 = u1, u3 = u1;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int ea = i * BS + lc * 17 + 4 * s4 + lg;  // R_ii^-1[lc][4 s4 + lg]
          const double ar = Ir[ea], ai = Ii[ea];
          u1 = mf(ar, tr[s4], u1);
          u2 = mf(ai, ti[s4], u2);
          u3 = mf(ar + ai, tr[s4] + ti[s4], u3);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ex = (16 * j + 4 * r + lg) * GS + 16 * i + lc;
          Gr[ex] = -(u1[r] - u2[r]);
          Gi[ex] = -(u3[r] - u1[r] - u2[r]);
        }
      }
      __syncthreads();
    }
  }
  // X to global, n x n row-major, zero below the diagonal
  cplx* Xb = X + (long)b * n * n;
  for (int e = tid; e < n * n; e += CQ_WAVES * 64) {
    const int r = e / n, c = e % n, rb = r >> 4, cb = c >> 4;
    cplx v = make_double2(0.0, 0.0);
    if (rb == cb) {
      const int ex = rb * BS + (r & 15) * 17 + (c & 15);
      v = make_double2(Ir[ex], Ii[ex]);
    } else if (rb < cb) {
      if (first_order) {
        v = make_double2(-Gr[r * GS + c], -Gi[r * GS + c]);
      } else {
        const int ex = (16 * cb + (r & 15)) * GS + 16 * rb + (c & 15);
        v = make_double2(Gr[ex], Gi[ex]);
      }
    }
    Xb[e] = v;
  }
  if (pass == 0 && tid == 0) flag[b] = 0;
}

template <int NB>
void launch_split(int batch, int m, int n, const MatView& S, cplx* Gp, int nparts, cplx* X, int* flag,
                  int pass, int drop, hipStream_t s) {
  hipLaunchKernelGGL((k_gram_part<NB>), dim3(nparts, batch), dim3(1024), 0, s, m, n, S, Gp, nparts);
  check(hipGetLastError(), "gram_part launch");
  const size_t shm = (size_t)CqL<NB>::TOTAL * sizeof(double);
  static const bool attr = [&]() {
    check(hipFuncSetAttribute((const void*)k_chol_inv<NB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shm),
          "chol_inv lds attribute");
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL((k_chol_inv<NB>), dim3(batch), dim3(CQ_WAVES * 64), shm, s, n, Gp, nparts, X, flag,
                     pass, drop);
  check(hipGetLastError(), "chol_inv launch");
}

void split_pass(int batch, int m, int n, const MatView& S, cplx* Gp, int nparts, cplx* X, int* flag, int pass,
                int drop, hipStream_t s) {
  switch ((n + 15) / 16) {
    case 2: launch_split<2>(batch, m, n, S, Gp, nparts, X, flag, pass, drop, s); break;
    case 3: launch_split<3>(batch, m, n, S, Gp, nparts, X, flag, pass, drop, s); break;
    case 4: launch_split<4>(batch, m, n, S, Gp, nparts, X, flag, pass, drop, s); break;
    default: launch_split<5>(batch, m, n, S, Gp, nparts, X, flag, pass, drop, s); break;
  }
}

// C = S X for every matrix of the batch on the library's GEMM
void split_product(int batch, int m, int n, const cplx* S, long lds, long sS, const cplx* X, cplx* C, long ldc,
                   long sC, cplx* gws, hipStream_t s) {
  GemmArgs g;
  g.M = m; g.N = n; g.K = n; g.opA = OP_N; g.opB = OP_N;
  g.A = S; g.lda = lds; g.sA1 = sS; g.sA2 = 0;
  g.B = X; g.ldb = n; g.sB1 = (long)n * n; g.sB2 = 0;
  g.C = C; g.ldc = ldc; g.sC1 = sC; g.sC2 = 0;
  g.nb1 = batch; g.nb2 = 1;
  g.alpha = make_double2(1.0, 0.0);
  g.beta = make_double2(0.0, 0.0);
  const int ks = gemm_ksplit(m, n, n, batch, false);
  if (ks > 1) {
    g.ws = gws;
    g.ksplit = ks;
  }
  gemm(g, s);
}

size_t split_gemm_ws(int batch, int m, int n) {
  const int ks = gemm_ksplit(m, n, n, batch, false);
  return ks > 1 ? (size_t)ks * batch * m * n : 0;
}

template <int NB>
void launch_cq(int batch, int m, int n, const MatView& A, const MatOut& Q, int* flag, int drop, hipStream_t s) {
  const size_t shm = (size_t)CqL<NB>::TOTAL * sizeof(double);
  // once per kernel and process (thread-safe static initialisation)
  static const bool attr = [&]() {
    check(hipFuncSetAttribute((const void*)k_cholqr2<NB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shm),
          "cholqr2 lds attribute");
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL((k_cholqr2<NB>), dim3(batch), dim3(CQ_WAVES * 64), shm, s, m, n, A, Q, flag, drop);
  check(hipGetLastError(), "cholqr2 launch");
}

}  // namespace

// shapes the fallback's register kernel holds too: up to 192 rows, 168
// beyond 64 columns
bool orth_ok(int m, int n) { return m >= n && n > 16 && n <= 80 && m > 32 && m <= (n > 64 ? 168 : CQ_MAXM); }

size_t orth_ws(int batch, int m, int n) {
  return (size_t)(batch + 3) / 4 + (size_t)batch * n * n + qr_ws(batch, m, n);
}

size_t orth_split_ws(int batch, int m, int n) {
  const int nparts = (m + GP_ROWS - 1) / GP_ROWS, NB = (n + 15) / 16, NT = NB * (NB + 1) / 2;
  return (size_t)(batch + 3) / 4 + (size_t)batch * nparts * NT * 256 + (size_t)batch * n * n +
         (size_t)batch * m * n + split_gemm_ws(batch, m, n) + (size_t)batch * n * n + qr_ws(batch, m, n);
}

bool orth_split(int batch, int m, int n, MatView A, MatOut Q, cplx* ws, hipStream_t s, bool drop) {
  if (batch <= 0) return true;
  if (!orth_ok(m, n) || A.cs != 1 || A.conj || Q.cs != 1) return false;
  const int nparts = (m + GP_ROWS - 1) / GP_ROWS, NB = (n + 15) / 16, NT = NB * (NB + 1) / 2;
  int* flag = (int*)ws;
  cplx* Gp = ws + (batch + 3) / 4;
  cplx* X = Gp + (size_t)batch * nparts * NT * 256;
  cplx* Q1 = X + (size_t)batch * n * n;
  cplx* gws = Q1 + (size_t)batch * m * n;
  cplx* Rs = gws + split_gemm_ws(batch, m, n);
  cplx* hws = Rs + (size_t)batch * n * n;
  // pass 0 on A, pass 1 on Q1 = A X
  split_pass(batch, m, n, A, Gp, nparts, X, flag, 0, drop, s);
  split_product(batch, m, n, A.base, A.rs, A.sb, X, Q1, n, (long)m * n, gws, s);
  split_pass(batch, m, n, MatView{Q1, (long)n, 1, (long)m * n, 0}, Gp, nparts, X, flag, 1, drop, s);
  split_product(batch, m, n, Q1, n, (long)m * n, X, Q.base, Q.rs, Q.sb, gws, s);
  // Householder for the flagged matrices (the others exit at once)
  const MatOut R{Rs, (long)n, 1, (long)n * n};
  if (!qr_2d_vectors(batch, m, n, A, R, hws, s, flag) || !qr_form_q(batch, m, n, Q, hws, s, flag))
    throw std::logic_error("orth: no Householder variant for the shape");
  return true;
}

bool orth(int batch, int m, int n, MatView A, MatOut Q, cplx* ws, hipStream_t s, bool drop) {
  if (batch <= 0) return true;
  if (!orth_ok(m, n)) return false;
  int* flag = (int*)ws;
  cplx* Rs = ws + (batch + 3) / 4;
  cplx* hws = Rs + (size_t)batch * n * n;
  switch ((n + 15) / 16) {
    case 2: launch_cq<2>(batch, m, n, A, Q, flag, drop, s); break;
    case 3: launch_cq<3>(batch, m, n, A, Q, flag, drop, s); break;
    case 4: launch_cq<4>(batch, m, n, A, Q, flag, drop, s); break;
    default: launch_cq<5>(batch, m, n, A, Q, flag, drop, s); break;
  }
  // Householder for the flagged matrices (the others exit at once)
  const MatOut R{Rs, (long)n, 1, (long)n * n};
  if (!qr_2d_vectors(batch, m, n, A, R, hws, s, flag) || !qr_form_q(batch, m, n, Q, hws, s, flag))
    throw std::logic_error("orth: no Householder variant for the shape");
  return true;
}

}  // namespace qtt
