// Blocked Householder QR for the sketched unfoldings of large ranks
// (m <= 320 rows, 96 < n <= 160 columns, m >= n), one workgroup per matrix.
//
// At rank cap 128 with oversampling 16 the left-to-right sweep of
// TT-rounding (Sec. 3, eq. rounding_condition_tt) orthonormalises
// Y_k = P_k W_{k+1} of 288 x 144 complex doubles: 663 KB, more than the
// 512 KB register file and the 160 KB LDS of a compute unit together hold
// as working set.  The matrix therefore lives in the workspace (global
// memory, L2-resident) in panel-major order, and one workgroup of 16 waves
// walks over its 16-column panels:
//
//  1. the panel is loaded into registers (wave w: rows [20 w, 20 w + 20),
//     lane l: column l % 16 at rows 20 w + l / 16 + 4 i, i < 5) and factored
//     column by column with one reflector rebuilt by every lane from the
//     published partial inner products (two barriers per column);
//  2. R rows of the panel columns are written, V (unit lower trapezoidal)
//     goes to LDS and to the workspace;
//  3. T of the compact WY form H = I - V T V^H, from the Gram V^H V on the
//     matrix cores and the recurrence T[0:j, j] = -tau_j T[0:j, 0:j]
//     (V^H V)[0:j, j];
//  4. every later panel c is updated by a wave of its own that streams the
//     panel's rows from L2 twice: W = V^H C over 4-row slices, W <- T^H W,
//     C <- C - V W over 16-row blocks, all on v_mfma_f64_16x16x4f64
//     (complex products as four real ones).
// Q (m x n) is formed afterwards by k_qr_formq2: one workgroup per
// 16-column group of Q applies the panels' block reflectors in reverse order
// from V and T in the workspace.
#include "fact_device.h"

#include <stdexcept>

namespace qtt {

namespace {

using namespace dev;

typedef double dv4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dv4 mfma(double a, double b, dv4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ cplx czero() { return make_double2(0.0, 0.0); }

constexpr int QB_WAVES = 16;                 // waves per workgroup
constexpr int QB_RPL = 5;                    // panel rows per lane
constexpr int QB_RW = 4 * QB_RPL;            // rows per wave (20)
constexpr int QB_MAXM = QB_WAVES * QB_RW;    // 320
constexpr int QB_MAXN = 160;
constexpr int QB_VST = 17;                   // LDS row stride of V (complex)
constexpr int QB_GW = 4;                     // waves forming the Gram V^H V

// workspace per matrix: V [np][m][16], T [np][16][16], tau [np][16] (the
// layout of qr_ws_per_matrix's blocked part), then the working matrix in
// panel-major order [nc][m][16]
__global__ __launch_bounds__(QB_WAVES * 64) void k_qr_big(int m, int n, MatView A, MatOut R,
                                                          cplx* ws, long wsz) {
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cl = lane & 15, rq = lane >> 4;
  const int base = w * QB_RW;
  const int k = min(m, n), np = (k + 15) / 16, nc = (n + 15) / 16;

  __shared__ cplx Vs[QB_MAXM * QB_VST];
  __shared__ cplx xbuf[2][QB_MAXM];
  __shared__ cplx part[QB_WAVES][16];
  __shared__ cplx rowj[16];
  __shared__ cplx taus[16], invs[16];
  __shared__ double betas[16];
  __shared__ cplx Ts[16][QB_VST];
  __shared__ cplx Gp[QB_GW][256];

  cplx* Vg = ws + (long)b * wsz;
  cplx* Tg = Vg + (long)np * m * 16;
  cplx* taug = Tg + (long)np * 256;
  cplx* Aw = taug + (long)np * 16;

  // working copy of A, panel-major, columns beyond n zero
  {
    const long total = (long)nc * m * 16;
    for (long e = tid; e < total; e += QB_WAVES * 64) {
      const int c = (int)(e / ((long)m * 16));
      const int r = (int)((e >> 4) % m);
      const int col = 16 * c + (int)(e & 15);
      Aw[e] = col < n ? ldv(A, b, r, col) : czero();
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int p = 0; p < np; ++p) {
    const int j0 = 16 * p, jn = min(k, j0 + 16);
    const int col = j0 + cl;
    const cplx* Cp = Aw + (long)p * m * 16;
    // the working matrix is re-read by waves other than the one that last
    // wrote it: drop this compute unit's vector L1 lines (agent-scope
    // acquire) so the reads see the stores in L2
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    cplx a[QB_RPL];
#pragma unroll
    for (int i = 0; i < QB_RPL; ++i) {
      const int row = base + rq + 4 * i;
      a[i] = csel(row < m, Cp[min(row, m - 1) * 16 + cl], czero());
    }
    if (cl == 0) {
#pragma unroll
      for (int i = 0; i < QB_RPL; ++i) {
        const int row = base + rq + 4 * i;
        xbuf[j0 & 1][row] = csel(row > j0 && row < m, a[i], czero());
      }
    }
    // ---- 1. panel factorisation ----
    for (int j = j0; j < jn; ++j) {
      const int xb = j & 1;
      __syncthreads();
      cplx pp = czero();
#pragma unroll
      for (int i = 0; i < QB_RPL; ++i) cdot_acc(pp, xbuf[xb][base + rq + 4 * i], a[i]);
      pp.x += __shfl_xor(pp.x, 16);
      pp.y += __shfl_xor(pp.y, 16);
      pp.x += __shfl_xor(pp.x, 32);
      pp.y += __shfl_xor(pp.y, 32);
      if (rq == 0) part[w][cl] = pp;
      if (j >= base && j < base + QB_RW && ((j - base - rq) & 3) == 0) {
        // the row-j entry of this lane's column (one-hot sum: an indexed
        // pick would move the register array to scratch)
        cplx r = czero();
#pragma unroll
        for (int i = 0; i < QB_RPL; ++i) {
          const double e = (base + rq + 4 * i == j) ? 1.0 : 0.0;
          r.x = fma(e, a[i].x, r.x);
          r.y = fma(e, a[i].y, r.y);
        }
        rowj[cl] = r;
      }
      __syncthreads();
      // sums of the 16 waves' partials, four loads in flight at a time (all
      // sixteen hoisted would spill the register budget of 1024 threads)
      double s = 0.0;
      cplx P = czero();
#pragma unroll 4
      for (int q = 0; q < QB_WAVES; ++q) {
        s += part[q][j - j0].x;
        P.x += part[q][cl].x;
        P.y += part[q][cl].y;
        if ((q & 3) == 3) asm volatile("" ::: "memory");
      }
      const cplx al = rowj[j - j0];
      const cplx rj = rowj[cl];
      cplx tau, inv;
      double beta;
      householder(al, s, tau, inv, beta);
      if (w == 0 && lane == 0) {
        taus[j - j0] = tau;
        invs[j - j0] = inv;
        betas[j - j0] = beta;
      }
      // v^H a_col = conj(inv) P + a[j][col]; a -= f v with v = x inv below
      // the diagonal and v_j = 1: a -= (f inv) x, a[j] -= f
      cplx f = czero(), g = czero();
      if (col > j && col < n) {
        const cplx cp = cmul(make_double2(inv.x, -inv.y), P);
        f = cmul(make_double2(tau.x, -tau.y), make_double2(cp.x + rj.x, cp.y + rj.y));
        g = cmul(f, inv);
      }
#pragma unroll
      for (int i = 0; i < QB_RPL; ++i) {
        const cplx x = xbuf[xb][base + rq + 4 * i];
        caxpy_sub(a[i], g, x);
        const double e = (base + rq + 4 * i == j) ? 1.0 : 0.0;
        a[i].x = fma(-e, f.x, a[i].x);
        a[i].y = fma(-e, f.y, a[i].y);
      }
      if (j + 1 < jn && col == j + 1) {
#pragma unroll
        for (int i = 0; i < QB_RPL; ++i) {
          const int row = base + rq + 4 * i;
          xbuf[xb ^ 1][row] = csel(row > j + 1 && row < m, a[i], czero());
        }
      }
    }
    __syncthreads();  // taus, invs, betas of the panel complete
    // ---- 2. R rows of the panel columns, V to LDS and workspace ----
    {
      cplx* vgp = Vg + (long)p * m * 16;
      const bool live = col < jn;
      const cplx ic = invs[cl];
      const double bc = betas[cl];
      cplx* Rb = R.base + b * R.sb;
#pragma unroll
      for (int i = 0; i < QB_RPL; ++i) {
        const int row = base + rq + 4 * i;
        const cplx v = cmul(a[i], ic);
        const bool lo = live && row > col && row < m, di = live && row == col;
        const cplx vv = make_double2(lo ? v.x : (di ? 1.0 : 0.0), lo ? v.y : 0.0);
        Vs[row * QB_VST + cl] = vv;
        if (row < m) vgp[row * 16 + cl] = vv;
        // R: the panel columns' rows above and on the diagonal, zero below
        if (row < k && col < n)
          Rb[(long)row * R.rs + (long)col * R.cs] =
              di ? make_double2(bc, 0.0) : csel(row < col, a[i], czero());
      }
      if (w == 0 && lane < 16) taug[(long)p * 16 + lane] = lane < jn - j0 ? taus[lane] : czero();
    }
    __syncthreads();
    // ---- 3. T: Gram V^H V over 4-row slices (V is zero above row j0) ----
    if (w < QB_GW) {
      dv4 gr = {0.0, 0.0, 0.0, 0.0}, gi = {0.0, 0.0, 0.0, 0.0};
      const int s0 = j0 / 4, s1 = (m + 3) / 4;
      for (int sl = s0 + w; sl < s1; sl += QB_GW) {
        const cplx v = Vs[(4 * sl + rq) * QB_VST + cl];
        gr = mfma(v.x, v.x, gr);
        gr = mfma(v.y, v.y, gr);
        gi = mfma(v.x, v.y, gi);
        gi = mfma(-v.y, v.x, gi);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) Gp[w][(4 * r + rq) * 16 + cl] = make_double2(gr[r], gi[r]);
    }
    __syncthreads();
    if (tid < 256) {
      cplx g = czero();
#pragma unroll
      for (int q = 1; q < QB_GW; ++q) {
        g.x += Gp[q][tid].x;
        g.y += Gp[q][tid].y;
      }
      Gp[0][tid] = make_double2(Gp[0][tid].x + g.x, Gp[0][tid].y + g.y);
    }
    __syncthreads();
    if (w == 0 && lane < 16) {
      // row i of T, column by column; the Ts row is written and read by
      // the same lane only
      const int i = lane, used = jn - j0;
      for (int j = 0; j < 16; ++j) {
        const cplx tj = taus[j];
        cplx acc = czero();
        for (int c = i; c < j; ++c) {
          const cplx t = Ts[i][c], g = Gp[0][c * 16 + j];
          acc.x += t.x * g.x - t.y * g.y;
          acc.y += t.x * g.y + t.y * g.x;
        }
        const cplx tn = cmul(make_double2(-tj.x, -tj.y), acc);
        const cplx t = j < used ? (i < j ? tn : (i == j ? tj : czero())) : czero();
        Ts[i][j] = t;
        Tg[(long)p * 256 + i * 16 + j] = t;
      }
    }
    __syncthreads();
    // ---- 4. later panels: C <- C - V T^H V^H C, one wave per panel ----
    const int c = p + 1 + w;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (c < nc) {
      cplx* Cc = Aw + (long)c * m * 16;
      dv4 wr = {0.0, 0.0, 0.0, 0.0}, wi = {0.0, 0.0, 0.0, 0.0};
      const int s0 = j0 / 4, s1 = (m + 3) / 4;
      // W = V^H C over 4-row slices, four slices of loads in flight
      for (int sl = s0; sl < s1; sl += 4) {
        cplx cv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int row = 4 * (sl + u) + rq;
          const cplx t = Cc[min(row, m - 1) * 16 + cl];
          cv[u] = csel(sl + u < s1 && row < m, t, czero());
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int row = 4 * (sl + u) + rq;
          const cplx v = Vs[min(row, QB_MAXM - 1) * QB_VST + cl];
          wr = mfma(v.x, cv[u].x, wr);
          wr = mfma(v.y, cv[u].y, wr);
          wi = mfma(v.x, cv[u].y, wi);
          wi = mfma(-v.y, cv[u].x, wi);
        }
      }
      // W2 = T^H W: A operand T^H[cl][4s + rq] = conj(T[4s + rq][cl])
      dv4 w2r = {0.0, 0.0, 0.0, 0.0}, w2i = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const cplx t = Ts[4 * s + rq][cl];
        w2r = mfma(t.x, wr[s], w2r);
        w2r = mfma(t.y, wi[s], w2r);
        w2i = mfma(t.x, wi[s], w2i);
        w2i = mfma(-t.y, wr[s], w2i);
      }
      // C <- C - V W2 over 16-row blocks (D layout: lane holds rows
      // 16 q + 4 r + rq, r < 4, of column cl)
      for (int q = j0 / 16; q < (m + 15) / 16; ++q) {
        dv4 dr, di;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * q + 4 * r + rq;
          const cplx t = Cc[min(row, m - 1) * 16 + cl];
          dr[r] = row < m ? t.x : 0.0;
          di[r] = row < m ? t.y : 0.0;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const cplx v = Vs[(16 * q + cl) * QB_VST + 4 * s + rq];
          dr = mfma(-v.x, w2r[s], dr);
          dr = mfma(v.y, w2i[s], dr);
          di = mfma(-v.x, w2i[s], di);
          di = mfma(-v.y, w2r[s], di);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * q + 4 * r + rq;
          if (row < m) Cc[row * 16 + cl] = make_double2(dr[r], di[r]);
        }
      }
    }
    // the stores of the update have reached L2 before the barrier
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();  // panel p + 1 updated before it is loaded
  }
}

// Q (m x k) from the panels' V and T in the workspace, one workgroup per
// 16-column group of Q (grid (batch, np)), RB waves of 4 RPL rows each.  The
// group holds its block of Q in registers in the MFMA D layout and meets
// the panels p <= its own in reverse order: W = V_p^H Q (row-block partials
// summed in LDS), W <- T_p W, Q <- Q - V_p W.
template <int RB, int RPL>
__global__ __launch_bounds__(RB * 64) void k_qr_formq2(int m, int n, MatOut Q, const cplx* ws, long wsz) {
  constexpr int NQ = RPL / 4, MR = RB * 4 * RPL, NT = RB * 64;
  const int b = blockIdx.x, cg = blockIdx.y, tid = threadIdx.x, lane = tid & 63;
  const int rb = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cl = lane & 15, rq = lane >> 4;
  const int col = cg * 16 + cl;
  const int base = rb * 4 * RPL;
  const int k = min(m, n), np = (k + 15) / 16;
  extern __shared__ cplx dyn[];
  cplx* Vs = dyn;              // [MR][QB_VST]
  cplx* Wp = dyn + MR * QB_VST;  // [RB][256]
  __shared__ cplx Ts[16][QB_VST];
  const cplx* Vg = ws + (long)b * wsz;
  const cplx* Tg = Vg + (long)np * m * 16;
  dv4 ar[NQ], ai[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = base + 16 * q + 4 * r + rq;
      ar[q][r] = (row == col && col < k) ? 1.0 : 0.0;
      ai[q][r] = 0.0;
    }
  for (int p = min(np - 1, cg); p >= 0; --p) {
    const int j0 = 16 * p;
    __syncthreads();  // the previous panel's Vs, Ts, Wp reads are done
    {
      constexpr int CNT = (MR * 16 + NT - 1) / NT;
      cplx t[CNT];
#pragma unroll
      for (int u = 0; u < CNT; ++u) {
        const int e = tid + u * NT, row = min(e >> 4, m - 1);
        t[u] = Vg[((long)p * m + row) * 16 + (e & 15)];
      }
      const cplx tt = Tg[(long)p * 256 + (tid & 255)];
#pragma unroll
      for (int u = 0; u < CNT; ++u) {
        const int e = tid + u * NT, row = e >> 4;
        if (e < MR * 16) Vs[row * QB_VST + (e & 15)] = csel(row < m, t[u], czero());
      }
      if (tid < 256) Ts[tid >> 4][tid & 15] = tt;
    }
    __syncthreads();
    // W partial = V^H Q over this wave's rows at or below j0
    {
      dv4 wr = {0.0, 0.0, 0.0, 0.0}, wi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = base + 16 * q + 4 * r;
          if (row + 3 < j0) continue;
          const cplx v = Vs[(row + rq) * QB_VST + cl];
          wr = mfma(v.x, ar[q][r], wr);
          wr = mfma(v.y, ai[q][r], wr);
          wi = mfma(v.x, ai[q][r], wi);
          wi = mfma(-v.y, ar[q][r], wi);
        }
#pragma unroll
      for (int r = 0; r < 4; ++r) Wp[rb * 256 + (4 * r + rq) * 16 + cl] = make_double2(wr[r], wi[r]);
    }
    __syncthreads();
    if (base + 4 * RPL > j0) {
      dv4 Wr = {0.0, 0.0, 0.0, 0.0}, Wi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < RB; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const cplx e = Wp[q * 256 + (4 * r + rq) * 16 + cl];
          Wr[r] += e.x;
          Wi[r] += e.y;
        }
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
      // Q <- Q - V W2 over the wave's 16-row blocks
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (base + 16 * q + 15 < j0) continue;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const cplx v = Vs[(base + 16 * q + cl) * QB_VST + 4 * s + rq];
          ar[q] = mfma(-v.x, w2r[s], ar[q]);
          ar[q] = mfma(v.y, w2i[s], ar[q]);
          ai[q] = mfma(-v.x, w2i[s], ai[q]);
          ai[q] = mfma(-v.y, w2r[s], ai[q]);
        }
      }
    }
  }
  cplx* Qb = Q.base + b * Q.sb;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = base + 16 * q + 4 * r + rq;
      if (row < m && col < k) Qb[(long)row * Q.rs + (long)col * Q.cs] = make_double2(ar[q][r], ai[q][r]);
    }
}

template <int RB, int RPL>
bool try_formq2(int batch, int m, int n, const MatOut& Q, const cplx* ws, long wsz, hipStream_t s) {
  constexpr int MR = RB * 4 * RPL;
  if (m > MR) return false;
  const int k = m < n ? m : n, np = (k + 15) / 16;
  const size_t shm = (size_t)(MR * QB_VST + RB * 256) * sizeof(cplx);
  static const bool attr = [&]() {
    check(hipFuncSetAttribute((const void*)k_qr_formq2<RB, RPL>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm),
          "qr_formq2 lds attribute");
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL((k_qr_formq2<RB, RPL>), dim3(batch, np), dim3(RB * 64), shm, s, m, n, Q, ws, wsz);
  check(hipGetLastError(), "qr_formq2 launch");
  return true;
}

}  // namespace

bool qr_big(int batch, int m, int n, MatView A, MatOut R, MatOut Q, cplx* ws, hipStream_t s) {
  if (batch <= 0 || m <= 0 || n <= 0) return true;
  if (m < n || m > QB_MAXM || n > QB_MAXN) return false;
  const long wsz = (long)qr_ws_per_matrix(m, n);
  hipLaunchKernelGGL(k_qr_big, dim3(batch), dim3(QB_WAVES * 64), 0, s, m, n, A, R, ws, wsz);
  check(hipGetLastError(), "qr_big launch");
  if (Q.base == nullptr) return true;
  // Q: row blocks of 32 rows (8 per lane)
  if (try_formq2<6, 8>(batch, m, n, Q, ws, wsz, s) || try_formq2<8, 8>(batch, m, n, Q, ws, wsz, s) ||
      try_formq2<10, 8>(batch, m, n, Q, ws, wsz, s))
    return true;
  throw std::logic_error("qr_big: Q formation shape");
}

}  // namespace qtt
