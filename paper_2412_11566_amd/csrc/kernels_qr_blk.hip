// Blocked Householder QR on the matrix cores, one workgroup per matrix, for
// the tall sketched unfoldings of TT-rounding (Sec. 3: the left-to-right
// sweep orthonormalises Y_k = P_k W_{k+1}, typically 160 x 80).
//
// Register layout: wave (rb, cg) holds rows [rb RBS, (rb + 1) RBS) of column
// group cg (16 columns); lane l holds column 16 cg + l % 16 at rows
// rb RBS + l / 16 + 4 i, i < RPL.  Four consecutive i form a 16 x 16 block
// laid out exactly as the D operand (and, per 4-row slice, the B operand)
// of v_mfma_f64_16x16x4f64, so block products need no data movement:
//   A operand: lane l holds A[l % 16][l / 16]
//   B operand: lane l holds B[l / 16][l % 16]
//   D:         lane l, register r holds D[4 r + l / 16][l % 16]
//
// Panel p (the 16 columns of group p):
//  1. the waves of group p factor the panel column by column (norms and
//     inner products: sums over the lane's rows, exchanges between the four
//     lane quarters, row blocks met in LDS); only these waves touch their
//     data during the 16 steps;
//  2. the panel's reflectors become one block reflector H = I - V T V^H
//     (compact WY form): V unit lower trapezoidal, and T upper triangular
//     from the recurrence T[0:j, j] = -tau_j T[0:j, 0:j] (V^H V)[0:j, j],
//     T[j, j] = tau_j, with V^H V computed on the matrix cores;
//  3. the waves of the later groups apply H^H to their columns with three
//     small block products on the matrix cores: W = V^H A, W <- T^H W,
//     A <- A - V W.
// Q = H_0 H_1 ... [I; 0] is formed afterwards in reverse panel order with
// the same block products (W = V^H Q, W <- T W, Q <- Q - V W) from V and T
// kept in the workspace; a column group of Q only meets the reflectors of
// panels at or before its own.  k_qr_formq1 forms Q alone (one workgroup
// per column group, T rebuilt in LDS from V and tau) after the unblocked
// register QR of kernels_fact.hip has written the vectors.
#include "fact_device.h"

#include <stdexcept>

namespace qtt {

namespace {

using namespace dev;

typedef double dv4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dv4 mfma(double a, double b, dv4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// row stride (complex entries) of the LDS copy of V: 17 keeps the column
// reads of the update step off a single bank group
constexpr int VST = 17;

// complex zero as a value (a named local would be kept in scratch memory
// across the compiler-only memory clobbers below)
__device__ __forceinline__ cplx cz() { return make_double2(0.0, 0.0); }

// bound the LDS loads kept in flight in the row loops (a compiler-only
// memory clobber; hoisting every row's load would spill the matrix)
#define QRB_WINDOW(i) \
  if (((i) & 3) == 3) asm volatile("" ::: "memory")

// a copy of a lane index the compiler cannot see through: address
// arithmetic built on it stays inside the loop iteration instead of being
// hoisted out of the loop and held in registers for its whole length
#define OPAQUE(dst, src) asm volatile("v_mov_b32 %0, %1" : "=v"(dst) : "v"(src))

// element i of the lane's rows (row base + rq + 4 i) in the real and
// imaginary register blocks: block i / 4, register i % 4
#define AR(i) ar[(i) >> 2][(i) & 3]
#define AI(i) ai[(i) >> 2][(i) & 3]

// W (D layout) <- V^H X over the wave's rows at or below row j0: A operand
// conj(V[row][cl]) with row = base + 4 i + rq, B operand X[row][col]
template <int RPL>
__device__ __forceinline__ void blk_vhx(const cplx* Vs, int base, int rq, int cl, int j0,
                                        const dv4 (&ar)[RPL / 4], const dv4 (&ai)[RPL / 4],
                                        dv4& wr, dv4& wi) {
  wr = dv4{0.0, 0.0, 0.0, 0.0};
  wi = dv4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    if (base + 4 * i + 3 < j0) continue;  // V is zero above row j0
    const cplx v = Vs[(base + 4 * i + rq) * VST + cl];
    wr = mfma(v.x, AR(i), wr);
    wr = mfma(v.y, AI(i), wr);
    wi = mfma(v.x, AI(i), wi);
    wi = mfma(-v.y, AR(i), wi);
    QRB_WINDOW(i);
  }
}

// X <- X - V W2 for the wave's 16-row blocks at or below row j0: A operand
// V[16 q + cl][4 s + rq], B operand register s of W2 (D layout)
template <int RPL>
__device__ __forceinline__ void blk_sub_vw(const cplx* Vs, int base, int rq, int cl, int j0,
                                           const dv4& w2r, const dv4& w2i, dv4 (&ar)[RPL / 4],
                                           dv4 (&ai)[RPL / 4]) {
#pragma unroll
  for (int q = 0; q < RPL / 4; ++q) {
    if (base + 16 * q + 15 < j0) continue;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const cplx v = Vs[(base + 16 * q + cl) * VST + 4 * s + rq];
      ar[q] = mfma(-v.x, w2r[s], ar[q]);
      ar[q] = mfma(v.y, w2i[s], ar[q]);
      ai[q] = mfma(-v.x, w2i[s], ai[q]);
      ai[q] = mfma(-v.y, w2r[s], ai[q]);
    }
    asm volatile("" ::: "memory");
  }
}

// W (D layout) = sum over row blocks of the partials of column group cg
template <int RB, int CG>
__device__ __forceinline__ void blk_wsum(const cplx* Wp, int cg, int rq, int cl, dv4& Wr, dv4& Wi) {
  Wr = dv4{0.0, 0.0, 0.0, 0.0};
  Wi = dv4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < RB; ++q) {
    const cplx* Wq = Wp + ((long)q * CG + cg) * 256;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const cplx e = Wq[(4 * r + rq) * 16 + cl];
      Wr[r] += e.x;
      Wi[r] += e.y;
    }
  }
}

// Q = H_0 ... H_{np-1} [I_k; 0] in reverse panel order from V_p and T_p in
// global memory: the column groups at or after panel p meet H_p as three
// block products on the matrix cores (W = V^H Q, W <- T W, Q <- Q - V W);
// a group before panel p is still a block of the identity, untouched by
// H_p.  The register arrays hold Q on return (also written to Q.base).
template <int RB, int RPL, int CG>
__device__ __forceinline__ void formq_phase(int m, int k, int np, int b, int tid, int rb, int cg,
                                            int cgl, int pstart, int cl0, int rq0, int col, int base,
                                            cplx* Vs, cplx* Wp, cplx (*Ts)[VST], const cplx* Vg,
                                            const cplx* Tg, MatOut Q, dv4 (&ar)[RPL / 4],
                                            dv4 (&ai)[RPL / 4]) {
  constexpr int RBS = 4 * RPL, MR = RB * RBS, NT = RB * CG * 64;
  const int rq = rq0;
  cplx* Qb = Q.base + b * Q.sb;
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int row = base + rq + 4 * i;
    AR(i) = (row == col && col < k) ? 1.0 : 0.0;
    AI(i) = 0.0;
  }
  for (int p = pstart; p >= 0; --p) {
    const int j0 = 16 * p;
    int rq, cl;
    OPAQUE(rq, rq0);
    OPAQUE(cl, cl0);
    __syncthreads();  // the previous panel's Vs, Ts, Wp reads are done
    {
      // every load of the panel issued before the LDS stores
      constexpr int CNT = (MR * 16 + NT - 1) / NT, TCNT = (256 + NT - 1) / NT;
      cplx t[CNT], tt[TCNT];
#pragma unroll
      for (int q = 0; q < CNT; ++q) {
        const int e = tid + q * NT, row = min(e >> 4, m - 1);
        t[q] = Vg[((long)p * m + row) * 16 + (e & 15)];
      }
#pragma unroll
      for (int q = 0; q < TCNT; ++q) tt[q] = Tg[(long)p * 256 + min(tid + q * NT, 255)];
#pragma unroll
      for (int q = 0; q < CNT; ++q) {
        const int e = tid + q * NT, row = e >> 4;
        if (e < MR * 16)
          Vs[row * VST + (e & 15)] = make_double2(row < m ? t[q].x : 0.0, row < m ? t[q].y : 0.0);
      }
#pragma unroll
      for (int q = 0; q < TCNT; ++q) {
        const int e = tid + q * NT;
        if (e < 256) Ts[e >> 4][e & 15] = tt[q];
      }
    }
    __syncthreads();
    const bool live = cg >= p;
    if (live) {
      dv4 wr, wi;
      blk_vhx<RPL>(Vs, base, rq, cl, j0, ar, ai, wr, wi);
      cplx* Wq = Wp + ((long)rb * CG + cgl) * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r) Wq[(4 * r + rq) * 16 + cl] = make_double2(wr[r], wi[r]);
    }
    __syncthreads();
    if (live && base + RBS > j0) {
      dv4 Wr, Wi;
      blk_wsum<RB, CG>(Wp, cgl, rq, cl, Wr, Wi);
      // W2 = T W: A operand T[cl][4s + rq]
      dv4 w2r = {0.0, 0.0, 0.0, 0.0}, w2i = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const cplx t = Ts[cl][4 * s + rq];
        w2r = mfma(t.x, Wr[s], w2r);
        w2r = mfma(-t.y, Wi[s], w2r);
        w2i = mfma(t.x, Wi[s], w2i);
        w2i = mfma(t.y, Wr[s], w2i);
      }
      blk_sub_vw<RPL>(Vs, base, rq, cl, j0, w2r, w2i, ar, ai);
    }
  }
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int row = base + rq + 4 * i;
    if (row < m && col < k)
      Qb[(long)row * Q.rs + (long)col * Q.cs] = make_double2(AR(i), AI(i));
    QRB_WINDOW(i);
  }
}

template <int RB, int RPL, int CG>
__global__ __launch_bounds__(RB * CG * 64) void k_qr_blk(int m, int n, MatView A, MatOut R,
                                                         MatOut Q, cplx* ws, long wsz) {
  static_assert(RPL % 4 == 0, "rows per lane come in 16-row blocks");
  constexpr int RBS = 4 * RPL, MR = RB * RBS, NQ = RPL / 4, NT = RB * CG * 64;
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rb = w / CG, cg = w % CG;
  const int cl0 = lane & 15, rq0 = lane >> 4;
  const int cl = cl0, rq = rq0;
  const int col = cg * 16 + cl;
  const int base = rb * RBS;
  const int k = min(m, n), np = (k + 15) / 16;

  extern __shared__ cplx dyn[];
  cplx* Vs = dyn;                        // [MR][VST]: V of the current panel
  cplx* Wp = dyn + MR * VST;             // [RB][CG][256]: per-row-block partials
  // xbuf holds the current column below its diagonal and zero elsewhere
  __shared__ cplx xbuf[2][MR];
  __shared__ cplx part[RB][16];
  __shared__ cplx rowj[16];
  __shared__ cplx taus[16], invs[16];
  __shared__ double betas[16];
  __shared__ cplx Ts[16][VST];

  cplx* Vg = ws + (long)b * wsz;        // [np][m][16]
  cplx* Tg = Vg + (long)np * m * 16;     // [np][16][16]

  dv4 ar[NQ], ai[NQ];
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int row = base + rq + 4 * i;
    const cplx v = (row < m && col < n) ? ldv(A, b, row, col) : cz();
    AR(i) = v.x;
    AI(i) = v.y;
    QRB_WINDOW(i);
  }

  for (int p = 0; p < np; ++p) {
    const int j0 = 16 * p, jn = min(k, j0 + 16);
    const bool panel = cg == p;  // wave-uniform
    int rq, cl;
    OPAQUE(rq, rq0);
    OPAQUE(cl, cl0);
    if (panel && col == j0) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = base + rq + 4 * i;
        const bool below = row > j0 && row < m;
        xbuf[j0 & 1][row] = make_double2(below ? AR(i) : 0.0, below ? AI(i) : 0.0);
      }
    }
    // ---- 1. panel factorisation (waves of group p) ----
    for (int j = j0; j < jn; ++j) {
      const int xb = j & 1;
      int rq, cl;
      OPAQUE(rq, rq0);
      OPAQUE(cl, cl0);
      const bool rowsLive = base + RBS > j;
      const bool holdsRowJ = j >= base && j < base + RBS;
      __syncthreads();
      if (panel) {
        cplx pp = cz();
        if (rowsLive) {
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            cdot_acc(pp, xbuf[xb][base + rq + 4 * i], make_double2(AR(i), AI(i)));
            QRB_WINDOW(i);
          }
        }
        pp.x += __shfl_xor(pp.x, 16);
        pp.y += __shfl_xor(pp.y, 16);
        pp.x += __shfl_xor(pp.x, 32);
        pp.y += __shfl_xor(pp.y, 32);
        if (rq == 0) part[rb][cl] = pp;
        if (holdsRowJ) {
          // one-hot sums (a compare-and-pick would index registers)
          cplx r = cz();
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            const double e = (base + rq + 4 * i == j) ? 1.0 : 0.0;
            r.x = fma(e, AR(i), r.x);
            r.y = fma(e, AI(i), r.y);
          }
          if (j - base - rq >= 0 && ((j - base - rq) & 3) == 0) rowj[cl] = r;
        }
      }
      __syncthreads();
      if (!panel) continue;
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < RB; ++q) s += part[q][j - j0].x;
      const cplx al = rowj[j - j0];
      cplx P = cz();
#pragma unroll
      for (int q = 0; q < RB; ++q) P = make_double2(P.x + part[q][cl].x, P.y + part[q][cl].y);
      const cplx rj = rowj[cl];
      cplx tau, inv;
      double beta;
      householder(al, s, tau, inv, beta);
      if (rb == 0 && lane == 0) {
        taus[j - j0] = tau;
        invs[j - j0] = inv;
        betas[j - j0] = beta;
      }
      if (rowsLive) {
        // v^H a_col = conj(inv) P + a[j][col];  a -= f v with v = x inv below
        // the diagonal and v_j = 1:  a -= (f inv) x,  a[j] -= f
        cplx f = cz(), g = cz();
        if (col > j && col < n) {
          const cplx cp = cmul(make_double2(inv.x, -inv.y), P);
          f = cmul(make_double2(tau.x, -tau.y), make_double2(cp.x + rj.x, cp.y + rj.y));
          g = cmul(f, inv);
        }
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const cplx x = xbuf[xb][base + rq + 4 * i];
          AR(i) = fma(-g.x, x.x, AR(i));
          AR(i) = fma(g.y, x.y, AR(i));
          AI(i) = fma(-g.x, x.y, AI(i));
          AI(i) = fma(-g.y, x.x, AI(i));
          QRB_WINDOW(i);
        }
        if (holdsRowJ) {
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            const double e = (base + rq + 4 * i == j) ? 1.0 : 0.0;
            AR(i) = fma(-e, f.x, AR(i));
            AI(i) = fma(-e, f.y, AI(i));
          }
        }
      }
      if (j + 1 < jn && col == j + 1) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int row = base + rq + 4 * i;
          const bool below = row > j + 1 && row < m;
          xbuf[xb ^ 1][row] = make_double2(below ? AR(i) : 0.0, below ? AI(i) : 0.0);
        }
      }
    }
    __syncthreads();  // taus, invs, betas of the panel complete
    // ---- 2. V and T of the panel ----
    if (panel) {
      cplx* vgp = Vg + (long)p * m * 16;
      const bool live = col < jn;
      const cplx ic = invs[cl];
      const double bc = betas[cl];
      dv4 gr = {0.0, 0.0, 0.0, 0.0}, gi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = base + rq + 4 * i;
        const cplx v = cmul(make_double2(AR(i), AI(i)), ic);
        // V: v below the diagonal, 1 on it, 0 above (and for columns
        // beyond k); the registers keep R on and above the diagonal
        const bool lo = live && row > col, di = live && row == col;
        const double vr = lo ? v.x : (di ? 1.0 : 0.0), vi = lo ? v.y : 0.0;
        AR(i) = lo ? v.x : (di ? bc : AR(i));
        AI(i) = lo ? v.y : (di ? 0.0 : AI(i));
        Vs[row * VST + cl] = make_double2(vr, vi);
        if (Q.base != nullptr && row < m) vgp[row * 16 + cl] = make_double2(vr, vi);
        // V^H V over this wave's rows: the lane's entry is both operands
        gr = mfma(vr, vr, gr);
        gr = mfma(vi, vi, gr);
        gi = mfma(vr, vi, gi);
        gi = mfma(-vi, vr, gi);
        QRB_WINDOW(i);
      }
      cplx* G = Wp + (long)rb * CG * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r) G[(4 * r + rq) * 16 + cl] = make_double2(gr[r], gi[r]);
    }
    __syncthreads();
    if (w == 0 && lane < 16) {
      // row `lane` of T, column by column (the Ts row is written and read
      // by the same lane only)
      const int i = lane;
      for (int j = 0; j < 16; ++j) {
        const cplx tj = taus[j];
        cplx t = cz();
        if (j < jn - j0) {
          if (i < j) {
            cplx acc = cz();
            for (int c = i; c < j; ++c) {
              cplx gcj = cz();
#pragma unroll
              for (int q = 0; q < RB; ++q) {
                const cplx gq = Wp[(long)q * CG * 256 + c * 16 + j];
                gcj.x += gq.x;
                gcj.y += gq.y;
              }
              const cplx tic = Ts[i][c];
              acc.x += tic.x * gcj.x - tic.y * gcj.y;
              acc.y += tic.x * gcj.y + tic.y * gcj.x;
            }
            t = cmul(make_double2(-tj.x, -tj.y), acc);
          } else if (i == j) {
            t = tj;
          }
        }
        Ts[i][j] = t;
        if (Q.base != nullptr) Tg[(long)p * 256 + i * 16 + j] = t;
      }
    }
    __syncthreads();
    // ---- 3. trailing groups: A <- A - V (T^H (V^H A)) ----
    const bool trail = cg > p;
    if (trail) {
      dv4 wr, wi;
      blk_vhx<RPL>(Vs, base, rq, cl, j0, ar, ai, wr, wi);
      cplx* Wq = Wp + ((long)rb * CG + cg) * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r) Wq[(4 * r + rq) * 16 + cl] = make_double2(wr[r], wi[r]);
    }
    __syncthreads();
    if (trail && base + RBS > j0) {
      dv4 Wr, Wi;
      blk_wsum<RB, CG>(Wp, cg, rq, cl, Wr, Wi);
      // W2 = T^H W: A operand T^H[cl][4s + rq] = conj(T[4s + rq][cl])
      dv4 w2r = {0.0, 0.0, 0.0, 0.0}, w2i = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const cplx t = Ts[4 * s + rq][cl];
        w2r = mfma(t.x, Wr[s], w2r);
        w2r = mfma(t.y, Wi[s], w2r);
        w2i = mfma(t.x, Wi[s], w2i);
        w2i = mfma(-t.y, Wr[s], w2i);
      }
      blk_sub_vw<RPL>(Vs, base, rq, cl, j0, w2r, w2i, ar, ai);
    }
  }

  cplx* Rb = R.base + b * R.sb;
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int row = base + rq + 4 * i;
    if (row < k && col < n)
      Rb[(long)row * R.rs + (long)col * R.cs] =
          make_double2(row <= col ? AR(i) : 0.0, row <= col ? AI(i) : 0.0);
    QRB_WINDOW(i);
  }
  if (Q.base == nullptr) return;
  formq_phase<RB, RPL, CG>(m, k, np, b, tid, rb, cg, cg, np - 1, cl0, rq0, col, base, Vs, Wp, Ts, Vg,
                           Tg, Q, ar, ai);
}

// Q alone from the panel vectors and T blocks in the workspace (the Q phase
// of k_qr_blk as its own kernel, after the unblocked register kernel has
// produced R and the vectors), with one workgroup per 16-column group of Q
// (grid (batch, np)): the groups are independent, so each runs on a compute
// unit of its own and applies only the panels p <= its group (a later panel
// leaves an identity block untouched); RB waves split the rows.
template <int RB, int RPL>
__global__ __launch_bounds__(RB * 64) void k_qr_formq1(int m, int n, MatOut Q, cplx* ws, long wsz,
                                                      const int* only) {
  constexpr int NQ = RPL / 4;
  const int b = blockIdx.x, cg = blockIdx.y, tid = threadIdx.x, lane = tid & 63;
  if (only != nullptr && only[b] == 0) return;
  const int rb = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cl0 = lane & 15, rq0 = lane >> 4;
  const int col = cg * 16 + cl0;
  const int base = rb * 4 * RPL;
  const int k = min(m, n), np = (k + 15) / 16;
  const int pmax = min(np - 1, cg);
  extern __shared__ cplx dyn[];
  cplx* Vs = dyn;
  cplx* Wp = dyn + RB * 4 * RPL * VST;
  cplx* Gl = Wp + RB * 256;  // Gram of panel p at Gl[p * 256], p <= pmax
  cplx* Tl = Gl + np * 256;  // T of panel p at Tl[p * 256]
  __shared__ cplx Ts[16][VST];
  const cplx* Vg = ws + (long)b * wsz;
  const cplx* taug = Vg + (long)np * m * 16 + (long)np * 256;
  // T of the panels p <= pmax this group meets (compact WY; each group
  // builds its own, in parallel with the other groups, instead of a launch
  // of its own): wave rb takes panels rb, rb + RB, ...; the Gram
  // V_p^H V_p on the matrix cores over 4-row slices from row 16 p (V is
  // zero above), then the recurrence T[i][j] = -tau_j sum_{c<j} T[i][c]
  // G[c][j], T[i][i] = tau_i, one row of T per lane
  {
    const int cl = lane & 15, rq = lane >> 4;
    const int nsl = (m + 3) / 4;
    for (int p = rb; p <= pmax; p += RB) {
      const cplx* V = Vg + (long)p * m * 16;
      dv4 gr = {0.0, 0.0, 0.0, 0.0}, gi = {0.0, 0.0, 0.0, 0.0};
      // up to 24 slices of loads in flight before their products
      for (int q0 = 4 * p; q0 < nsl; q0 += 24) {
        cplx v[24];
#pragma unroll
        for (int q = 0; q < 24; ++q) {
          const int row = 4 * (q0 + q) + rq;
          const cplx t = V[(long)min(row, m - 1) * 16 + cl];
          v[q] = make_double2(row < m ? t.x : 0.0, row < m ? t.y : 0.0);
        }
#pragma unroll
        for (int q = 0; q < 24; ++q) {
          gr = mfma(v[q].x, v[q].x, gr);
          gr = mfma(v[q].y, v[q].y, gr);
          gi = mfma(v[q].x, v[q].y, gi);
          gi = mfma(-v[q].y, v[q].x, gi);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) Gl[p * 256 + (4 * r + rq) * 16 + cl] = make_double2(gr[r], gi[r]);
    }
    __syncthreads();
    for (int p = rb; p <= pmax; p += RB) {
      if (lane < 16) {
        const int i = lane;
        const cplx* G = Gl + p * 256;
        const cplx* tau = taug + (long)p * 16;
        cplx t[16], tv[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) tv[j] = tau[j];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const cplx tj = tv[j];
          cplx acc = cz();
#pragma unroll
          for (int c = 0; c < j; ++c) {
            const cplx g = G[c * 16 + j];
            acc.x += t[c].x * g.x - t[c].y * g.y;
            acc.y += t[c].x * g.y + t[c].y * g.x;
          }
          const cplx tn = cmul(make_double2(-tj.x, -tj.y), acc);
          t[j] = i < j ? tn : (i == j ? tj : cz());
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) Tl[p * 256 + i * 16 + j] = t[j];
      }
    }
    __syncthreads();
  }
  dv4 ar[NQ], ai[NQ];
  formq_phase<RB, RPL, 1>(m, k, np, b, tid, rb, cg, 0, pmax, cl0, rq0, col, base, Vs, Wp, Ts, Vg, Tl,
                          Q, ar, ai);
}

#undef AR
#undef AI

template <int RB, int RPL>
bool try_qr_formq1(int batch, int m, int n, const MatOut& Q, cplx* ws, hipStream_t s, const int* only) {
  constexpr int MR = RB * 4 * RPL;
  const int k = m < n ? m : n, np = (k + 15) / 16;
  if (m > MR) return false;
  // V rows, W partials, and the Gram and T of up to np panels
  const size_t shm = (size_t)(MR * VST + RB * 256 + 2 * 6 * 256) * sizeof(cplx);
  if (np > 6) return false;
  static const bool attr = [&]() {
    check(hipFuncSetAttribute((const void*)k_qr_formq1<RB, RPL>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm),
          "qr_formq1 lds attribute");
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL((k_qr_formq1<RB, RPL>), dim3(batch, np), dim3(RB * 64), shm, s, m, n, Q, ws,
                     (long)qr_ws_per_matrix(m, n), only);
  check(hipGetLastError(), "qr_formq1 launch");
  return true;
}

// row blocks of 4 RPL rows: 4 waves up to 128 rows, then 5 or 6 waves of
// 32 rows (measured at 160 x 80 and 160 x 64 against 2, 4 and 10 waves)
bool qr_formq_split(int batch, int m, int n, const MatOut& Q, cplx* ws, hipStream_t s, const int* only) {
  return try_qr_formq1<4, 4>(batch, m, n, Q, ws, s, only) || try_qr_formq1<4, 8>(batch, m, n, Q, ws, s, only) ||
         try_qr_formq1<5, 8>(batch, m, n, Q, ws, s, only) || try_qr_formq1<6, 8>(batch, m, n, Q, ws, s, only);
}

template <int RB, int RPL, int CG>
bool try_qr_blk(int batch, int m, int n, const MatView& A, const MatOut& R, const MatOut& Q,
                cplx* ws, hipStream_t s) {
  constexpr int MR = RB * 4 * RPL;
  if (m > MR || n > 16 * CG) return false;
  const long k = m < n ? m : n, np = (k + 15) / 16;
  // per-matrix slice of the qr() workspace
  const long wsz = (long)qr_ws_per_matrix(m, n);
  if (np * (16L * m + 256 + 16) > wsz) return false;
  const size_t shm = (size_t)(MR * VST + RB * CG * 256) * sizeof(cplx);
  // once per kernel and process (thread-safe static initialisation: the
  // load-case groups of a solve launch from several host threads)
  static const bool attr = [&]() {
    check(hipFuncSetAttribute((const void*)k_qr_blk<RB, RPL, CG>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm),
          "qr_blk lds attribute");
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL((k_qr_blk<RB, RPL, CG>), dim3(batch), dim3(RB * CG * 64), shm, s, m, n, A, R, Q,
                     ws, wsz);
  check(hipGetLastError(), "qr_blk launch");
  return true;
}

template <int CG>
bool qr_blk_cg(int batch, int m, int n, const MatView& A, const MatOut& R, const MatOut& Q, cplx* ws,
               hipStream_t s) {
  return try_qr_blk<2, 4, CG>(batch, m, n, A, R, Q, ws, s) ||
         try_qr_blk<2, 8, CG>(batch, m, n, A, R, Q, ws, s) ||
         try_qr_blk<2, 12, CG>(batch, m, n, A, R, Q, ws, s) ||
         try_qr_blk<2, 16, CG>(batch, m, n, A, R, Q, ws, s) ||
         try_qr_blk<2, 20, CG>(batch, m, n, A, R, Q, ws, s) ||
         try_qr_blk<2, 24, CG>(batch, m, n, A, R, Q, ws, s);
}

}  // namespace

bool qr_form_q(int batch, int m, int n, MatOut Q, cplx* ws, hipStream_t s, const int* only) {
  if (batch <= 0 || m <= 0 || n <= 0) return true;
  if (m < n || n <= 16 || n > 96 || m > 192) return false;
  return qr_formq_split(batch, m, n, Q, ws, s, only);
}

bool qr_blocked(int batch, int m, int n, MatView A, MatOut R, MatOut Q, cplx* ws, hipStream_t s) {
  if (batch <= 0 || m <= 0 || n <= 0) return true;
  if (m < n || n <= 16 || m > 192) return false;
  switch ((n + 15) / 16) {
    case 2: return qr_blk_cg<2>(batch, m, n, A, R, Q, ws, s);
    case 3: return qr_blk_cg<3>(batch, m, n, A, R, Q, ws, s);
    case 4: return qr_blk_cg<4>(batch, m, n, A, R, Q, ws, s);
    case 5: return qr_blk_cg<5>(batch, m, n, A, R, Q, ws, s);
    case 6: return qr_blk_cg<6>(batch, m, n, A, R, Q, ws, s);
    default: return false;
  }
}

}  // namespace qtt
