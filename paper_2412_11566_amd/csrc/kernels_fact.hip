// Latency-optimised factorisation kernels for the small matrices of
// TT-rounding (one workgroup per matrix, batch = trains processed together):
//
//  * k_qr_reg: Householder QR with the matrix held in registers.  Lane l of
//    every wave owns columns l, l + 64, ...; wave w owns a block of rows.
//    Reflector norms and dot products are reduced first over the wave's
//    rows (in registers) and then across the 8 waves through LDS; the
//    reflector itself is broadcast through LDS.
//  * k_jacobi_lds: one-sided Jacobi (Hestenes) on a square matrix resident
//    in LDS; 16 lanes cooperate on a column pair with shuffle reductions,
//    column norms are carried analytically within a sweep and recomputed
//    at its start.
#include "fact_device.h"

#include <stdexcept>

namespace qtt {

namespace {

using namespace dev;

// QNW waves per workgroup; wave w holds rows [w*RPW, (w+1)*RPW), lane l
// holds columns l + 64*c, c < CPL.
template <int QNW, int RPW, int CPL>
__global__ __launch_bounds__(QNW * 64) void k_qr_reg(int m, int n, MatView A, MatOut R, MatOut Q,
                                                    cplx* ws) {
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int k = min(m, n);
  cplx* V = ws + (long)b * ((long)m * k + k);
  __shared__ cplx vsh[QNW * RPW];
  __shared__ cplx part[QNW][64 * CPL];
  __shared__ double pn[QNW];
  __shared__ cplx sh_alpha, sh_tau, sh_inv;
  __shared__ double sh_beta;
  __shared__ cplx taus[64 * CPL];

  const int row0 = w * RPW;
  cplx a[RPW][CPL];
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int row = row0 + i, col = lane + 64 * c;
      a[i][c] = (row < m && col < n) ? ldv(A, b, row, col) : make_double2(0.0, 0.0);
    }

  for (int j = 0; j < k; ++j) {
    const int jl = j & 63, jc = j >> 6;
    if (lane == jl) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        if (c != jc) continue;
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          const int row = row0 + i;
          if (row > j && row < m) s += cabs2(a[i][c]);
          if (row == j) sh_alpha = a[i][c];
        }
      }
      pn[w] = s;
    }
    __syncthreads();
    if (tid == 0) {
      double xn2 = 0.0;
#pragma unroll
      for (int q = 0; q < QNW; ++q) xn2 += pn[q];
      const cplx alpha = sh_alpha;
      cplx tau, inv;
      double beta;
      householder(alpha, xn2, tau, inv, beta);
      sh_tau = tau;
      sh_inv = inv;
      sh_beta = beta;
      taus[j] = sh_tau;
      V[(long)m * k + j] = sh_tau;
    }
    __syncthreads();
    const cplx tj = sh_tau;
    if (tj.x == 0.0 && tj.y == 0.0) continue;
    const cplx inv = sh_inv;
    const double beta = sh_beta;
    if (lane == jl) {
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        if (c != jc) continue;
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          const int row = row0 + i;
          if (row > j && row < m) {
            a[i][c] = cmul(a[i][c], inv);
            vsh[row] = a[i][c];
            V[(long)j * m + row] = a[i][c];
          } else if (row == j) {
            vsh[row] = make_double2(1.0, 0.0);
            a[i][c] = make_double2(beta, 0.0);
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int col = lane + 64 * c;
      if (col > j && col < n) {
        cplx s = make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          const int row = row0 + i;
          if (row >= j && row < m) {
            const cplx t = cdotc(vsh[row], a[i][c]);
            s = make_double2(s.x + t.x, s.y + t.y);
          }
        }
        part[w][col] = s;
      }
    }
    __syncthreads();
    const cplx ctj = make_double2(tj.x, -tj.y);
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int col = lane + 64 * c;
      if (col > j && col < n) {
        cplx tot = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < QNW; ++q) tot = make_double2(tot.x + part[q][col].x, tot.y + part[q][col].y);
        const cplx f = cmul(ctj, tot);
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          const int row = row0 + i;
          if (row >= j && row < m) {
            const cplx fv = cmul(f, vsh[row]);
            a[i][c] = make_double2(a[i][c].x - fv.x, a[i][c].y - fv.y);
          }
        }
      }
    }
  }
  // R (k x n, upper trapezoidal)
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int row = row0 + i, col = lane + 64 * c;
      if (row < k && col < n)
        R.base[b * R.sb + (long)row * R.rs + (long)col * R.cs] =
            (row <= col) ? a[i][c] : make_double2(0.0, 0.0);
    }
  if (Q.base == nullptr) return;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int row = row0 + i, col = lane + 64 * c;
      a[i][c] = make_double2((row == col && col < k && row < m) ? 1.0 : 0.0, 0.0);
    }
  for (int j = k - 1; j >= 0; --j) {
    const cplx tj = taus[j];
    if (tj.x == 0.0 && tj.y == 0.0) continue;
    for (int r = j + tid; r < m; r += QNW * 64)
      vsh[r] = (r == j) ? make_double2(1.0, 0.0) : V[(long)j * m + r];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int col = lane + 64 * c;
      if (col >= j && col < k) {
        cplx s = make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          const int row = row0 + i;
          if (row >= j && row < m) {
            const cplx t = cdotc(vsh[row], a[i][c]);
            s = make_double2(s.x + t.x, s.y + t.y);
          }
        }
        part[w][col] = s;
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int col = lane + 64 * c;
      if (col >= j && col < k) {
        cplx tot = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < QNW; ++q) tot = make_double2(tot.x + part[q][col].x, tot.y + part[q][col].y);
        const cplx f = cmul(tj, tot);
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          const int row = row0 + i;
          if (row >= j && row < m) {
            const cplx fv = cmul(f, vsh[row]);
            a[i][c] = make_double2(a[i][c].x - fv.x, a[i][c].y - fv.y);
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int row = row0 + i, col = lane + 64 * c;
      if (row < m && col < k) Q.base[b * Q.sb + (long)row * Q.rs + (long)col * Q.cs] = a[i][c];
    }
}

template <int QNW, int RPW, int CPL>
bool try_qr(int batch, int m, int n, const MatView& A, const MatOut& R, const MatOut& Q, cplx* ws,
            hipStream_t s) {
  if (m > QNW * RPW || n > 64 * CPL) return false;
  hipLaunchKernelGGL((k_qr_reg<QNW, RPW, CPL>), dim3(batch), dim3(QNW * 64), 0, s, m, n, A, R, Q, ws);
  check(hipGetLastError(), "qr_reg launch");
  return true;
}


// Register QR, transposed layout: lane l holds rows l + 64*i (i < RPL),
// wave w holds columns w*CPW + c (c < CPW).  Column norms and reflector
// dot products are 64-lane shuffle reductions inside one wave.
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int RPL, int CPW, bool WANTQ>
__global__ __launch_bounds__(512) void k_qr_rows(int m, int n, MatView A, MatOut R, MatOut Q,
                                                 cplx* ws) {
  constexpr int NW = 8;
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int k = min(m, n);
  cplx* V = ws + (long)b * ((long)m * k + k);
  __shared__ cplx vsh[64 * RPL];
  __shared__ cplx taus[NW * CPW];
  const int col0 = w * CPW;
  cplx a[RPL][CPW];
#pragma unroll
  for (int i = 0; i < RPL; ++i)
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int row = lane + 64 * i, col = col0 + c;
      a[i][c] = (row < m && col < n) ? ldv(A, b, row, col) : make_double2(0.0, 0.0);
    }
  for (int j = 0; j < k; ++j) {
    const int jw = j / CPW, jc = j - jw * CPW;
    if (w == jw) {
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        if (c != jc) continue;
        double s = 0.0;
        cplx al = make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int row = lane + 64 * i;
          if (row > j && row < m) s += cabs2(a[i][c]);
          if (row == j) al = a[i][c];
        }
        s = wsum(s);
        al.x = wsum(al.x);
        al.y = wsum(al.y);
        cplx tau, inv;
        double beta;
        householder(al, s, tau, inv, beta);
        const bool zero = (tau.x == 0.0 && tau.y == 0.0);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int row = lane + 64 * i;
          if (row < m) {
            if (row > j) {
              if (!zero) a[i][c] = cmul(a[i][c], inv);
              vsh[row] = zero ? make_double2(0.0, 0.0) : a[i][c];
              V[(long)j * m + row] = vsh[row];
            } else if (row == j) {
              vsh[row] = make_double2(1.0, 0.0);
              a[i][c] = make_double2(beta, 0.0);
            }
          }
        }
        if (lane == 0) {
          taus[j - 0] = tau;
          V[(long)m * k + j] = tau;
        }
      }
    }
    __syncthreads();
    const cplx tj = taus[j];
    if (!(tj.x == 0.0 && tj.y == 0.0)) {
      cplx v[RPL];
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = lane + 64 * i;
        v[i] = (row >= j && row < m) ? vsh[row] : make_double2(0.0, 0.0);
      }
      const cplx ctj = make_double2(tj.x, -tj.y);
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int col = col0 + c;
        if (col <= j || col >= n) continue;
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const cplx t = cdotc(v[i], a[i][c]);
          sx += t.x;
          sy += t.y;
        }
        sx = wsum(sx);
        sy = wsum(sy);
        const cplx f = cmul(ctj, make_double2(sx, sy));
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const cplx fv = cmul(f, v[i]);
          a[i][c] = make_double2(a[i][c].x - fv.x, a[i][c].y - fv.y);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < RPL; ++i)
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int row = lane + 64 * i, col = col0 + c;
      if (row < k && col < n)
        R.base[b * R.sb + (long)row * R.rs + (long)col * R.cs] =
            (row <= col) ? a[i][c] : make_double2(0.0, 0.0);
    }
  if (!WANTQ || Q.base == nullptr) return;
#pragma unroll
  for (int i = 0; i < RPL; ++i)
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int row = lane + 64 * i, col = col0 + c;
      a[i][c] = make_double2((row == col && col < k && row < m) ? 1.0 : 0.0, 0.0);
    }
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    const cplx tj = taus[j];
    if (tj.x == 0.0 && tj.y == 0.0) continue;
    cplx v[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = lane + 64 * i;
      v[i] = (row < m && row > j) ? V[(long)j * m + row]
                                  : make_double2(row == j ? 1.0 : 0.0, 0.0);
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int col = col0 + c;
      if (col < j || col >= k) continue;
      double sx = 0.0, sy = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const cplx t = cdotc(v[i], a[i][c]);
        sx += t.x;
        sy += t.y;
      }
      sx = wsum(sx);
      sy = wsum(sy);
      const cplx f = cmul(tj, make_double2(sx, sy));
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const cplx fv = cmul(f, v[i]);
        a[i][c] = make_double2(a[i][c].x - fv.x, a[i][c].y - fv.y);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < RPL; ++i)
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int row = lane + 64 * i, col = col0 + c;
      if (row < m && col < k) Q.base[b * Q.sb + (long)row * Q.rs + (long)col * Q.cs] = a[i][c];
    }
}

// ---------------------------------------------------------------------------
// Householder QR with one workgroup barrier per column.
//
// Wave w owns rows [w*RPW, (w+1)*RPW); lane l owns columns l + 64 c
// (c < CPL).  Step j: every wave broadcasts column j of its own rows inside
// the wave (wave-private LDS) and forms partial inner products
// sum_r conj(x_r) a[r][col] over its rows r > j for every column; the wave
// holding row j publishes that row.  After the single barrier every thread
// sums the partials and rebuilds the same reflector (norm, beta, tau) from
// them, so the reflector needs no broadcast of its own.  Partials and row j
// are double-buffered across steps, which makes one barrier per step
// sufficient.  Q is then accumulated in place (Q = H_0 ... H_{k-1} [I; 0])
// from the reflectors left below the diagonal, again one barrier per step.
template <int NW, int RPW, int CPL>
__global__ __launch_bounds__(NW * 64) void k_qr_lc(int m, int n, MatView A, MatOut R, MatOut Q) {
  constexpr int NC = 64 * CPL;
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  // wave index as a scalar: branches on it stay uniform (no divergent
  // merges that would keep two copies of the register-resident matrix)
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int k = min(m, n);
  __shared__ cplx part[2][NW][NC];
  __shared__ cplx rowj[2][NC];
  __shared__ cplx colb[NW][RPW];
  __shared__ cplx taus[NC];
  const int row0 = w * RPW;
  cplx a[RPW][CPL];
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int row = row0 + i, col = lane + 64 * c;
      a[i][c] = (row < m && col < n) ? ldv(A, b, row, col) : make_double2(0.0, 0.0);
    }

  for (int j = 0; j < k; ++j) {
    const int buf = j & 1, jl = j & 63, jc = j >> 6;
    const bool live = row0 + RPW > j;  // this wave still has rows >= j
    if (live) {
      if (lane == jl) {
        // static register indices only (a select between columns would
        // turn `a` into an indexed array in scratch memory)
#pragma unroll
        for (int c = 0; c < CPL; ++c)
          if (jc == c) {
#pragma unroll
            for (int i = 0; i < RPW; ++i) colb[w][i] = a[i][c];
          }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      cplx p[CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) p[c] = make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        const int row = row0 + i;
        if (row > j && row < m) {
          const cplx x = colb[w][i];
#pragma unroll
          for (int c = 0; c < CPL; ++c) cdot_acc(p[c], x, a[i][c]);
        }
        if (row == j) {
#pragma unroll
          for (int c = 0; c < CPL; ++c) rowj[buf][lane + 64 * c] = a[i][c];
        }
      }
#pragma unroll
      for (int c = 0; c < CPL; ++c) part[buf][w][lane + 64 * c] = p[c];
    } else {
#pragma unroll
      for (int c = 0; c < CPL; ++c) part[buf][w][lane + 64 * c] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    // the reflector, rebuilt identically by every thread
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) s += part[buf][q][j].x;
    const cplx al = rowj[buf][j];
    cplx tau, inv;
    double beta;
    householder(al, s, tau, inv, beta);
    if (tid == 0) taus[j] = tau;
    if (!live) continue;
    // f_col = conj(tau) * v^H a_col, with v_j = 1 and v_r = x_r * inv
    const cplx cinv = make_double2(inv.x, -inv.y), ctau = make_double2(tau.x, -tau.y);
    cplx f[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int col = lane + 64 * c;
      f[c] = make_double2(0.0, 0.0);
      if (col > j && col < n) {
        cplx P = make_double2(0.0, 0.0);
#pragma unroll 4
        for (int q = 0; q < NW; ++q) P = make_double2(P.x + part[buf][q][col].x, P.y + part[buf][q][col].y);
        const cplx cp = cmul(cinv, P);
        const cplx rj = rowj[buf][col];
        f[c] = cmul(ctau, make_double2(cp.x + rj.x, cp.y + rj.y));
      }
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int row = row0 + i;
      if (row < j || row >= m) continue;
      const cplx v = (row == j) ? make_double2(1.0, 0.0) : cmul(colb[w][i], inv);
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int col = lane + 64 * c;
        if (col > j) {
          caxpy_sub(a[i][c], f[c], v);
        } else if (col == j) {
          a[i][c] = (row == j) ? make_double2(beta, 0.0) : v;
        }
      }
      // keep the scheduler from hoisting every row's LDS read (register
      // pressure would force the matrix into scratch)
      if ((i & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
  }
  // R (k x n, upper trapezoidal)
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int row = row0 + i, col = lane + 64 * c;
      if (row < k && col < n)
        R.base[b * R.sb + (long)row * R.rs + (long)col * R.cs] =
            (row <= col) ? a[i][c] : make_double2(0.0, 0.0);
    }
  if (Q.base == nullptr) return;
  // in-place accumulation: clear the upper part (R is written out), keep
  // the reflectors below the diagonal; columns >= k are not part of Q
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int row = row0 + i, col = lane + 64 * c;
      if (row <= col || col >= k) a[i][c] = make_double2(0.0, 0.0);
    }
  __syncthreads();  // taus complete
  for (int j = k - 1; j >= 0; --j) {
    const int buf = j & 1, jl = j & 63, jc = j >> 6;
    const bool live = row0 + RPW > j;
    const cplx tj = taus[j];
    if (live) {
      // column j: publish v (rows > j), then turn it into e_j
      if (lane == jl) {
#pragma unroll
        for (int c = 0; c < CPL; ++c)
          if (jc == c) {
#pragma unroll
            for (int i = 0; i < RPW; ++i) {
              colb[w][i] = a[i][c];
              a[i][c] = make_double2(row0 + i == j ? 1.0 : 0.0, 0.0);
            }
          }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      cplx p[CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) p[c] = make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        const int row = row0 + i;
        if (row < j || row >= m) continue;
        const cplx v = (row == j) ? make_double2(1.0, 0.0) : colb[w][i];
#pragma unroll
        for (int c = 0; c < CPL; ++c) cdot_acc(p[c], v, a[i][c]);
      }
#pragma unroll
      for (int c = 0; c < CPL; ++c) part[buf][w][lane + 64 * c] = p[c];
    } else {
#pragma unroll
      for (int c = 0; c < CPL; ++c) part[buf][w][lane + 64 * c] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (!live || (tj.x == 0.0 && tj.y == 0.0)) continue;
    cplx f[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int col = lane + 64 * c;
      cplx P = make_double2(0.0, 0.0);
      if (col >= j && col < k) {
#pragma unroll 4
        for (int q = 0; q < NW; ++q) P = make_double2(P.x + part[buf][q][col].x, P.y + part[buf][q][col].y);
      }
      f[c] = cmul(tj, P);
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int row = row0 + i;
      if (row < j || row >= m) continue;
      const cplx v = (row == j) ? make_double2(1.0, 0.0) : colb[w][i];
#pragma unroll
      for (int c = 0; c < CPL; ++c) caxpy_sub(a[i][c], f[c], v);
      if ((i & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int row = row0 + i, col = lane + 64 * c;
      if (row < m && col < k) Q.base[b * Q.sb + (long)row * Q.rs + (long)col * Q.cs] = a[i][c];
    }
}

// ---------------------------------------------------------------------------
// Householder QR over a 2D wave grid with quad reductions.
//
// Wave (rb, cg) holds row block rb (4*RPL rows) of column group cg (16
// columns); inside the wave lane l = rs + 4*cl holds column cg*16 + cl at
// rows rb*4*RPL + rs + 4*i, i < RPL.  The four lanes of a quad hold the same
// column, so a column's inner product over the wave's rows is an in-lane
// sum plus two DPP quad exchanges; row blocks meet in LDS.  A column group
// whose columns are all factored drops out of the loop, so the trailing
// work shrinks with j.  Step j: [barrier] partial inner products with
// x = column j (published in LDS by its owners) [barrier] every thread
// rebuilds the reflector from the partials, updates its columns, and the
// owners of column j+1 publish it.  Q is accumulated in place afterwards
// (Q = H_0 ... H_{k-1} [I; 0]) with the same two barriers per step.
// bound the LDS loads kept in flight inside the row loops to a window of 4
// rows (a compiler-only memory clobber; hoisting every row's load would
// spill the register-resident matrix)
#define QR2D_WINDOW(i) \
  if (((i) & 3) == 3) asm volatile("" ::: "memory")

__device__ __forceinline__ double dpp_xor1(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double dpp_xor2(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x4E, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x4E, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double dpp_half_mirror(double v) {   // lane i <- lane 7 - i (per 8)
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x141, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x141, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double dpp_mirror(double v) {        // lane i <- lane 15 - i (per 16)
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x140, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x140, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// sum over the 16 lanes of a DPP row, returned to every lane of the row
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_xor1(v);
  v += dpp_xor2(v);
  v += dpp_half_mirror(v);
  v += dpp_mirror(v);
  return v;
}
__device__ __forceinline__ cplx quad_sum(cplx p) {
  p.x += dpp_xor1(p.x);
  p.y += dpp_xor1(p.y);
  p.x += dpp_xor2(p.x);
  p.y += dpp_xor2(p.y);
  return p;
}

template <int RB, int RPL, int CG>
__global__ __launch_bounds__(RB * CG * 64) void k_qr_2d(int m, int n, MatView A, MatOut R, MatOut Q,
                                                        cplx* vout, long vsz, const int* only) {
  constexpr int NC = 16 * CG, RBS = 4 * RPL, MR = RB * RBS;
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  // only the matrices whose flag is set (the CholeskyQR kernel's fallbacks)
  if (only != nullptr && only[b] == 0) return;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rb = w / CG, cg = w % CG;
  const int rs = lane & 3, cl = lane >> 2;
  const int col = cg * 16 + cl;
  const int base = rb * RBS;  // first row of this wave's block
  const int k = min(m, n);
  __shared__ cplx part[RB][NC];
  __shared__ cplx rowj[NC];
  // xbuf holds the published column for the rows strictly below the
  // diagonal of the current step and zero elsewhere, so the inner loops
  // run branch-free over every row of the block
  __shared__ cplx xbuf[2][MR];
  __shared__ cplx taus[NC], invs[NC];
  __shared__ double betas[NC];
  cplx a[RPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int row = base + rs + 4 * i;
    a[i] = (row < m && col < n) ? ldv(A, b, row, col) : make_double2(0.0, 0.0);
    QR2D_WINDOW(i);
  }
  const cplx zero = make_double2(0.0, 0.0);
  if (col == 0) {
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = base + rs + 4 * i;
      xbuf[0][row] = csel(row > 0 && row < m, a[i], zero);
    }
  }
  for (int j = 0; j < k; ++j) {
    const int xb = j & 1, jg = j >> 4;
    const bool colsLive = cg >= jg;          // uniform
    const bool rowsLive = base + RBS > j;    // uniform: block has rows >= j
    const bool holdsRowJ = j >= base && j < base + RBS;
    __syncthreads();
    if (colsLive) {
      cplx p = zero;
      if (rowsLive) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          cdot_acc(p, xbuf[xb][base + rs + 4 * i], a[i]);
          QR2D_WINDOW(i);
        }
      }
      p = quad_sum(p);
      if (rs == 0) part[rb][col] = p;
      if (holdsRowJ) {
        // one-hot sums instead of a compare-and-pick: a pick lets the
        // compiler form a computed register index (scratch memory)
        cplx r = zero;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const double e = (base + rs + 4 * i == j) ? 1.0 : 0.0;
          r.x = fma(e, a[i].x, r.x);
          r.y = fma(e, a[i].y, r.y);
        }
        if (j - base - rs >= 0 && ((j - base - rs) & 3) == 0) rowj[col] = r;
      }
    }
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < RB; ++q) s += part[q][j].x;
    const cplx al = rowj[j];
    cplx tau, inv;
    double beta;
    householder(al, s, tau, inv, beta);
    if (tid == 0) {
      taus[j] = tau;
      invs[j] = inv;
      betas[j] = beta;
    }
    if (colsLive && rowsLive) {
      // v^H a_col = conj(inv) P + a[j][col];  a -= f v with v = x inv below
      // the diagonal and v_j = 1:  a -= (f inv) x,  a[j] -= f
      cplx f = zero, g = zero;
      if (col > j && col < n) {
        cplx P = zero;
#pragma unroll
        for (int q = 0; q < RB; ++q) P = make_double2(P.x + part[q][col].x, P.y + part[q][col].y);
        const cplx cp = cmul(make_double2(inv.x, -inv.y), P);
        const cplx rj = rowj[col];
        f = cmul(make_double2(tau.x, -tau.y), make_double2(cp.x + rj.x, cp.y + rj.y));
        g = cmul(f, inv);
      }
      // column j itself is left as x (f = g = 0 there); it becomes beta and
      // v = x inv in one pass after the loop
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        caxpy_sub(a[i], g, xbuf[xb][base + rs + 4 * i]);
        QR2D_WINDOW(i);
      }
      if (holdsRowJ) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const double e = (base + rs + 4 * i == j) ? 1.0 : 0.0;
          a[i].x = fma(-e, f.x, a[i].x);
          a[i].y = fma(-e, f.y, a[i].y);
        }
      }
    }
    // owners of column j + 1 publish it below its diagonal
    if (j + 1 < k && col == j + 1) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = base + rs + 4 * i;
        xbuf[xb ^ 1][row] = csel(row > j + 1 && row < m, a[i], zero);
      }
    }
  }
  __syncthreads();  // betas, invs complete
  if (col < k) {
    const cplx ic = invs[col];
    const double bc = betas[col];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = base + rs + 4 * i;
      const cplx v = cmul(a[i], ic);
      a[i] = csel(row > col, v, csel(row == col, make_double2(bc, 0.0), a[i]));
    }
  }
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int row = base + rs + 4 * i;
    if (row < k && col < n)
      R.base[b * R.sb + (long)row * R.rs + (long)col * R.cs] = csel(row <= col, a[i], zero);
    QR2D_WINDOW(i);
  }
  if (vout != nullptr) {
    // Householder vectors of 16-column panels for the matrix-core Q
    // formation: V[p][row][c] (unit diagonal, zero above), then tau[p][c]
    // after the T blocks
    const int np = (k + 15) / 16;
    cplx* V = vout + (long)b * vsz;
    if (col < np * 16) {  // columns of the last panel beyond k: zero
      cplx* vp = V + (long)(col >> 4) * m * 16 + (col & 15);
      const bool live = col < k;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = base + rs + 4 * i;
        if (row < m)
          vp[row * 16] = csel(live && row > col, a[i],
                              make_double2(live && row == col ? 1.0 : 0.0, 0.0));
        QR2D_WINDOW(i);
      }
    }
    if (tid < np * 16) {
      const int c = tid;
      V[(long)np * m * 16 + (long)np * 256 + c] = csel(c < k, taus[c], zero);
    }
    return;
  }
  if (Q.base == nullptr) return;
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int row = base + rs + 4 * i;
    if (row <= col || col >= k) a[i] = zero;
  }
  for (int j = k - 1; j >= 0; --j) {
    const int xb = j & 1, jg = j >> 4;
    const bool colsLive = cg >= jg;
    const bool rowsLive = base + RBS > j;
    const bool holdsRowJ = j >= base && j < base + RBS;
    // column j: publish v below the diagonal, then turn it into e_j (the
    // register update is a select, not a divergent branch)
    if (cg == jg) {
      const bool isJ = col == j;
      if (isJ) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int row = base + rs + 4 * i;
          xbuf[xb][row] = csel(row > j && row < m, a[i], zero);
        }
      }
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = base + rs + 4 * i;
        a[i] = csel(isJ, make_double2(row == j ? 1.0 : 0.0, 0.0), a[i]);
      }
    }
    __syncthreads();
    if (colsLive) {
      cplx p = zero;
      if (rowsLive) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          cdot_acc(p, xbuf[xb][base + rs + 4 * i], a[i]);
          QR2D_WINDOW(i);
        }
        if (holdsRowJ) {
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            const double e = (base + rs + 4 * i == j) ? 1.0 : 0.0;
            p.x = fma(e, a[i].x, p.x);
            p.y = fma(e, a[i].y, p.y);
          }
        }
      }
      p = quad_sum(p);
      if (rs == 0) part[rb][col] = p;
    }
    __syncthreads();
    const cplx tj = taus[j];
    if (!colsLive || !rowsLive || (tj.x == 0.0 && tj.y == 0.0)) continue;
    cplx f = zero;
    if (col >= j && col < k) {
      cplx P = zero;
#pragma unroll
      for (int q = 0; q < RB; ++q) P = make_double2(P.x + part[q][col].x, P.y + part[q][col].y);
      f = cmul(tj, P);
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      caxpy_sub(a[i], f, xbuf[xb][base + rs + 4 * i]);
      QR2D_WINDOW(i);
    }
    if (holdsRowJ) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const double e = (base + rs + 4 * i == j) ? 1.0 : 0.0;
        a[i].x = fma(-e, f.x, a[i].x);
        a[i].y = fma(-e, f.y, a[i].y);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int row = base + rs + 4 * i;
    if (row < m && col < k) Q.base[b * Q.sb + (long)row * Q.rs + (long)col * Q.cs] = a[i];
    QR2D_WINDOW(i);
  }
}

// The same algorithm with CPL columns per lane (lane l of wave (rb, cg)
// holds columns cg*16*CPL + l/4 + 16 c, c < CPL): every published value of
// the current column read from LDS serves CPL columns, which divides the
// LDS traffic of the two row loops (the bound of the one-column form) by
// CPL for the same register footprint per lane.
template <int RB, int RPL, int CG, int CPL>
__global__ __launch_bounds__(RB * CG * 64) void k_qr_2c(int m, int n, MatView A, MatOut R, MatOut Q) {
  constexpr int GW = 16 * CPL, NC = GW * CG, RBS = 4 * RPL, MR = RB * RBS;
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rb = w / CG, cg = w % CG;
  const int rs = lane & 3, cl = lane >> 2;
  const int col0 = cg * GW + cl;   // column of c = 0; column c is col0 + 16 c
  const int base = rb * RBS;
  const int k = min(m, n);
  __shared__ cplx part[RB][NC];
  __shared__ cplx rowj[NC];
  __shared__ cplx xbuf[2][MR];
  __shared__ cplx taus[NC], invs[NC];
  __shared__ double betas[NC];
  cplx a[CPL][RPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c)
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = base + rs + 4 * i, col = col0 + 16 * c;
      a[c][i] = (row < m && col < n) ? ldv(A, b, row, col) : make_double2(0.0, 0.0);
      QR2D_WINDOW(i);
    }
  const cplx zero = make_double2(0.0, 0.0);
  if (col0 == 0) {
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = base + rs + 4 * i;
      xbuf[0][row] = csel(row > 0 && row < m, a[0][i], zero);
    }
  }
  for (int j = 0; j < k; ++j) {
    const int xb = j & 1, jg = j / GW;
    const bool colsLive = cg >= jg;          // uniform
    const bool rowsLive = base + RBS > j;    // uniform
    const bool holdsRowJ = j >= base && j < base + RBS;
    __syncthreads();
    if (colsLive) {
      cplx p[CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) p[c] = zero;
      if (rowsLive) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const cplx x = xbuf[xb][base + rs + 4 * i];
#pragma unroll
          for (int c = 0; c < CPL; ++c) cdot_acc(p[c], x, a[c][i]);
          QR2D_WINDOW(i);
        }
      }
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        p[c] = quad_sum(p[c]);
        if (rs == 0) part[rb][col0 + 16 * c] = p[c];
      }
      if (holdsRowJ) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          cplx r = zero;
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            const double e = (base + rs + 4 * i == j) ? 1.0 : 0.0;
            r.x = fma(e, a[c][i].x, r.x);
            r.y = fma(e, a[c][i].y, r.y);
          }
          if (j - base - rs >= 0 && ((j - base - rs) & 3) == 0) rowj[col0 + 16 * c] = r;
        }
      }
    }
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < RB; ++q) s += part[q][j].x;
    const cplx al = rowj[j];
    cplx tau, inv;
    double beta;
    householder(al, s, tau, inv, beta);
    if (tid == 0) {
      taus[j] = tau;
      invs[j] = inv;
      betas[j] = beta;
    }
    if (colsLive && rowsLive) {
      cplx f[CPL], g[CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int col = col0 + 16 * c;
        f[c] = zero;
        g[c] = zero;
        if (col > j && col < n) {
          cplx P = zero;
#pragma unroll
          for (int q = 0; q < RB; ++q) P = make_double2(P.x + part[q][col].x, P.y + part[q][col].y);
          const cplx cp = cmul(make_double2(inv.x, -inv.y), P);
          const cplx rj = rowj[col];
          f[c] = cmul(make_double2(tau.x, -tau.y), make_double2(cp.x + rj.x, cp.y + rj.y));
          g[c] = cmul(f[c], inv);
        }
      }
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const cplx x = xbuf[xb][base + rs + 4 * i];
#pragma unroll
        for (int c = 0; c < CPL; ++c) caxpy_sub(a[c][i], g[c], x);
        QR2D_WINDOW(i);
      }
      if (holdsRowJ) {
#pragma unroll
        for (int c = 0; c < CPL; ++c)
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            const double e = (base + rs + 4 * i == j) ? 1.0 : 0.0;
            a[c][i].x = fma(-e, f[c].x, a[c][i].x);
            a[c][i].y = fma(-e, f[c].y, a[c][i].y);
          }
      }
    }
    // owners of column j + 1 publish it below its diagonal
    if (j + 1 < k) {
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        if (col0 + 16 * c != j + 1) continue;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int row = base + rs + 4 * i;
          xbuf[xb ^ 1][row] = csel(row > j + 1 && row < m, a[c][i], zero);
        }
      }
    }
  }
  __syncthreads();  // betas, invs complete
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int col = col0 + 16 * c;
    if (col < k) {
      const cplx ic = invs[col];
      const double bc = betas[col];
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = base + rs + 4 * i;
        const cplx v = cmul(a[c][i], ic);
        a[c][i] = csel(row > col, v, csel(row == col, make_double2(bc, 0.0), a[c][i]));
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CPL; ++c)
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = base + rs + 4 * i, col = col0 + 16 * c;
      if (row < k && col < n)
        R.base[b * R.sb + (long)row * R.rs + (long)col * R.cs] = csel(row <= col, a[c][i], zero);
      QR2D_WINDOW(i);
    }
  if (Q.base == nullptr) return;
#pragma unroll
  for (int c = 0; c < CPL; ++c)
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = base + rs + 4 * i, col = col0 + 16 * c;
      if (row <= col || col >= k) a[c][i] = zero;
    }
  for (int j = k - 1; j >= 0; --j) {
    const int xb = j & 1, jg = j / GW;
    const bool colsLive = cg >= jg;
    const bool rowsLive = base + RBS > j;
    const bool holdsRowJ = j >= base && j < base + RBS;
    // column j: publish v below the diagonal, then turn it into e_j
    if (cg == jg) {
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const bool isJ = col0 + 16 * c == j;
        if (isJ) {
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            const int row = base + rs + 4 * i;
            xbuf[xb][row] = csel(row > j && row < m, a[c][i], zero);
          }
        }
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int row = base + rs + 4 * i;
          a[c][i] = csel(isJ, make_double2(row == j ? 1.0 : 0.0, 0.0), a[c][i]);
        }
      }
    }
    __syncthreads();
    if (colsLive) {
      cplx p[CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) p[c] = zero;
      if (rowsLive) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const cplx x = xbuf[xb][base + rs + 4 * i];
#pragma unroll
          for (int c = 0; c < CPL; ++c) cdot_acc(p[c], x, a[c][i]);
          QR2D_WINDOW(i);
        }
        if (holdsRowJ) {
#pragma unroll
          for (int c = 0; c < CPL; ++c)
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
              const double e = (base + rs + 4 * i == j) ? 1.0 : 0.0;
              p[c].x = fma(e, a[c][i].x, p[c].x);
              p[c].y = fma(e, a[c][i].y, p[c].y);
            }
        }
      }
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        p[c] = quad_sum(p[c]);
        if (rs == 0) part[rb][col0 + 16 * c] = p[c];
      }
    }
    __syncthreads();
    const cplx tj = taus[j];
    if (!colsLive || !rowsLive || (tj.x == 0.0 && tj.y == 0.0)) continue;
    cplx f[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int col = col0 + 16 * c;
      f[c] = zero;
      if (col >= j && col < k) {
        cplx P = zero;
#pragma unroll
        for (int q = 0; q < RB; ++q) P = make_double2(P.x + part[q][col].x, P.y + part[q][col].y);
        f[c] = cmul(tj, P);
      }
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const cplx x = xbuf[xb][base + rs + 4 * i];
#pragma unroll
      for (int c = 0; c < CPL; ++c) caxpy_sub(a[c][i], f[c], x);
      QR2D_WINDOW(i);
    }
    if (holdsRowJ) {
#pragma unroll
      for (int c = 0; c < CPL; ++c)
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const double e = (base + rs + 4 * i == j) ? 1.0 : 0.0;
          a[c][i].x = fma(-e, f[c].x, a[c][i].x);
          a[c][i].y = fma(-e, f[c].y, a[c][i].y);
        }
    }
  }
#pragma unroll
  for (int c = 0; c < CPL; ++c)
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = base + rs + 4 * i, col = col0 + 16 * c;
      if (row < m && col < k) Q.base[b * Q.sb + (long)row * Q.rs + (long)col * Q.cs] = a[c][i];
      QR2D_WINDOW(i);
    }
}

template <int RB, int RPL, int CG, int CPL>
bool try_qr_2c(int batch, int m, int n, const MatView& A, const MatOut& R, const MatOut& Q,
               hipStream_t s) {
  if (m > RB * 4 * RPL || n > 16 * CPL * CG) return false;
  hipLaunchKernelGGL((k_qr_2c<RB, RPL, CG, CPL>), dim3(batch), dim3(RB * CG * 64), 0, s, m, n, A, R, Q);
  check(hipGetLastError(), "qr_2c launch");
  return true;
}

// Householder QR with one wave per group of 16 columns holding every row of
// its columns (lane l: column 16 cg + l / 4, rows l % 4 + 4 i, i < RPL).
// A column's inner products then reduce inside its wave (quad DPP), and
// every wave rebuilds the reflector itself from the published column
// (norm and leading entry read from LDS), so one barrier per column
// suffices: the owners of column j + 1 publish it after their update of
// step j.  Writes R and, when vout is given, the Householder vectors and
// tau per 16-column panel (the layout of the matrix-core Q formation).
template <int RPL, int CG>
__global__ __launch_bounds__(CG * 64) void k_qr_1r(int m, int n, MatView A, MatOut R, cplx* vout, long vsz) {
  constexpr int NC = 16 * CG, MR = 4 * RPL;
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int cg = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rs = lane & 3, cl = lane >> 2;
  const int col = cg * 16 + cl;
  const int k = min(m, n);
  // xbuf: the current column, every row (zero at rows >= m)
  __shared__ cplx xbuf[2][MR];
  __shared__ cplx taus[NC], invs[NC];
  __shared__ double betas[NC];
  const cplx zero = make_double2(0.0, 0.0);
  cplx a[RPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int row = rs + 4 * i;
    a[i] = (row < m && col < n) ? ldv(A, b, row, col) : make_double2(0.0, 0.0);
    QR2D_WINDOW(i);
  }
  if (col == 0) {
#pragma unroll
    for (int i = 0; i < RPL; ++i) xbuf[0][rs + 4 * i] = a[i];
  }
  for (int j = 0; j < k; ++j) {
    const int xb = j & 1;
    __syncthreads();
    if (cg < (j >> 4)) continue;  // every column of this wave is factored
    // inner product of x (rows below j) with this lane's column and |x|^2
    cplx p = zero;
    double sx = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = rs + 4 * i;
      const cplx xr = xbuf[xb][row];
      const cplx x = csel(row > j, xr, zero);
      cdot_acc(p, x, a[i]);
      sx = fma(x.x, x.x, fma(x.y, x.y, sx));
      QR2D_WINDOW(i);
    }
    // a[j][col]: the lane of the quad that holds row j contributes it
    cplx rj = zero;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const double e = (rs + 4 * i == j) ? 1.0 : 0.0;
      rj.x = fma(e, a[i].x, rj.x);
      rj.y = fma(e, a[i].y, rj.y);
    }
    p = quad_sum(p);
    rj = quad_sum(rj);
    sx += dpp_xor1(sx);
    sx += dpp_xor2(sx);
    const cplx al = xbuf[xb][j];
    cplx tau, inv;
    double beta;
    householder(al, sx, tau, inv, beta);
    if (col == j && rs == 0) {
      taus[j] = tau;
      invs[j] = inv;
      betas[j] = beta;
    }
    // v^H a_col = conj(inv) p + a[j][col];  a -= f v with v = x inv below
    // the diagonal and v_j = 1:  a -= (f inv) x,  a[j] -= f
    cplx f = zero, g = zero;
    if (col > j && col < n) {
      const cplx cp = cmul(make_double2(inv.x, -inv.y), p);
      f = cmul(make_double2(tau.x, -tau.y), make_double2(cp.x + rj.x, cp.y + rj.y));
      g = cmul(f, inv);
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = rs + 4 * i;
      const cplx xr = xbuf[xb][row];
      caxpy_sub(a[i], g, csel(row > j, xr, zero));
      const double e = (row == j) ? 1.0 : 0.0;
      a[i].x = fma(-e, f.x, a[i].x);
      a[i].y = fma(-e, f.y, a[i].y);
      QR2D_WINDOW(i);
    }
    if (j + 1 < k && col == j + 1) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) xbuf[xb ^ 1][rs + 4 * i] = a[i];
    }
  }
  __syncthreads();  // betas, invs, taus complete
  if (col < k) {
    const cplx ic = invs[col];
    const double bc = betas[col];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = rs + 4 * i;
      const cplx v = cmul(a[i], ic);
      a[i] = csel(row > col, v, csel(row == col, make_double2(bc, 0.0), a[i]));
    }
  }
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int row = rs + 4 * i;
    if (row < k && col < n)
      R.base[b * R.sb + (long)row * R.rs + (long)col * R.cs] = csel(row <= col, a[i], zero);
    QR2D_WINDOW(i);
  }
  if (vout == nullptr) return;
  const int np = (k + 15) / 16;
  cplx* V = vout + (long)b * vsz;
  if (col < np * 16) {
    cplx* vp = V + (long)(col >> 4) * m * 16 + (col & 15);
    const bool live = col < k;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = rs + 4 * i;
      if (row < m)
        vp[row * 16] = csel(live && row > col, a[i], make_double2(live && row == col ? 1.0 : 0.0, 0.0));
      QR2D_WINDOW(i);
    }
  }
  if (tid < np * 16) V[(long)np * m * 16 + (long)np * 256 + tid] = csel(tid < k, taus[tid], zero);
}

template <int RPL, int CG>
bool try_qr_1r(int batch, int m, int n, const MatView& A, const MatOut& R, cplx* vout, hipStream_t s) {
  if (m > 4 * RPL || n > 16 * CG) return false;
  hipLaunchKernelGGL((k_qr_1r<RPL, CG>), dim3(batch), dim3(CG * 64), 0, s, m, n, A, R, vout,
                     (long)qr_ws_per_matrix(m, n));
  check(hipGetLastError(), "qr_1r launch");
  return true;
}

template <int CG>
bool qr_1r_any(int batch, int m, int n, const MatView& A, const MatOut& R, cplx* vout, hipStream_t s) {
  return try_qr_1r<8, CG>(batch, m, n, A, R, vout, s) || try_qr_1r<16, CG>(batch, m, n, A, R, vout, s) ||
         try_qr_1r<24, CG>(batch, m, n, A, R, vout, s) || try_qr_1r<32, CG>(batch, m, n, A, R, vout, s) ||
         try_qr_1r<40, CG>(batch, m, n, A, R, vout, s);
}

// one-wave-per-column-group kernel for R (and the panel vectors), n <= 96,
// m <= 160
bool qr_1r_dispatch(int batch, int m, int n, const MatView& A, const MatOut& R, cplx* vout,
                    hipStream_t s) {
  switch ((n + 15) / 16) {
    case 2: return qr_1r_any<2>(batch, m, n, A, R, vout, s);
    case 3: return qr_1r_any<3>(batch, m, n, A, R, vout, s);
    case 4: return qr_1r_any<4>(batch, m, n, A, R, vout, s);
    case 5: return qr_1r_any<5>(batch, m, n, A, R, vout, s);
    case 6: return qr_1r_any<6>(batch, m, n, A, R, vout, s);
    default: return false;
  }
}

template <int RB, int RPL, int CG>
bool try_qr_2d(int batch, int m, int n, const MatView& A, const MatOut& R, const MatOut& Q,
               hipStream_t s, cplx* vout = nullptr, const int* only = nullptr) {
  if (m > RB * 4 * RPL || n > 16 * CG) return false;
  hipLaunchKernelGGL((k_qr_2d<RB, RPL, CG>), dim3(batch), dim3(RB * CG * 64), 0, s, m, n, A, R, Q, vout,
                     (long)qr_ws_per_matrix(m, n), only);
  check(hipGetLastError(), "qr_2d launch");
  return true;
}

template <int NW, int RPW, int CPL>
bool try_qr_lc(int batch, int m, int n, const MatView& A, const MatOut& R, const MatOut& Q,
               hipStream_t s) {
  if (m > NW * RPW || n > 64 * CPL) return false;
  hipLaunchKernelGGL((k_qr_lc<NW, RPW, CPL>), dim3(batch), dim3(NW * 64), 0, s, m, n, A, R, Q);
  check(hipGetLastError(), "qr_lc launch");
  return true;
}

template <int RPL, int CPW, bool WANTQ = true>
bool try_qr_rows(int batch, int m, int n, const MatView& A, const MatOut& R, const MatOut& Q, cplx* ws,
                 hipStream_t s) {
  if (m > 64 * RPL || n > 8 * CPW) return false;
  if (WANTQ != (Q.base != nullptr) && !WANTQ) return false;
  hipLaunchKernelGGL((k_qr_rows<RPL, CPW, WANTQ>), dim3(batch), dim3(512), 0, s, m, n, A, R, Q, ws);
  check(hipGetLastError(), "qr_rows launch");
  return true;
}

// ---------------------------------------------------------------------------
constexpr int JNT = 1024;
constexpr int JMAXN = 96;

typedef double jdv4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ jdv4 jmf(double a, double b, jdv4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Whether any column pair of the n x n column-major LDS matrix W (column
// stride ld) still needs a rotation: |x_a^H x_b|^2 > tol^2 |x_a|^2 |x_b|^2
// with both norms above 1e-300, the test of the rotation loop, for all
// pairs at once.  The Gram blocks (I <= J) come from the matrix cores, one
// 16 x 16 block per wave at a time, three real products per complex K-step
// of 4 rows.  A sweep that would find no such pair changes nothing, so this
// replaces the last, rotation-free sweep (79 rounds at n = 80, each
// streaming the whole matrix through LDS) by one pass over it.  Every wave
// must call it.
__device__ __forceinline__ bool jac_pairs_left(int n, int ld, const cplx* Wl, const double* nrm2,
                                               double tol) {
  const int tid = threadIdx.x, lane = tid & 63, lc = lane & 15, lg = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nb = (n + 15) >> 4, nt = nb * (nb + 1) / 2;
  bool hit = false;
  for (int t = w; t < nt; t += JNT / 64) {
    int I = 0, tt = t;
    while (tt >= nb - I) {
      tt -= nb - I;
      ++I;
    }
    const int J = I + tt;
    const int cI = 16 * I + lc, cJ = 16 * J + lc;
    jdv4 p1 = {0.0, 0.0, 0.0, 0.0}, p2 = p1, p3 = p1;
    for (int k0 = 0; k0 < n; k0 += 4) {
      const int row = k0 + lg;
      const cplx a = (row < n && cI < n) ? Wl[cI * ld + row] : make_double2(0.0, 0.0);
      const cplx c = (row < n && cJ < n) ? Wl[cJ * ld + row] : make_double2(0.0, 0.0);
      p1 = jmf(a.x, c.x, p1);
      p2 = jmf(-a.y, c.y, p2);
      p3 = jmf(a.x - a.y, c.x + c.y, p3);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ca = 16 * I + 4 * r + lg, cb = 16 * J + lc;
      if (ca < cb && cb < n) {
        const double gr = p1[r] - p2[r], gi = p3[r] - p1[r] - p2[r];
        const double al = nrm2[ca], be = nrm2[cb];
        if (gr * gr + gi * gi > tol * tol * (al * be) && al >= 1e-300 && be >= 1e-300) hit = true;
      }
    }
  }
  return hit;
}

__global__ __launch_bounds__(JNT) void k_jacobi_lds(int n, MatView A, MatOut U, double* S) {
  // n x n, column-major with column stride n + 1: the check of all pairs
  // reads 16 columns at one row per lane group, which a stride of n would
  // put in one LDS bank (n = 80: 1280 B)
  extern __shared__ cplx Wl[];
  __shared__ double nrm2[JMAXN];
  __shared__ double sig[JMAXN];
  __shared__ int rankpos[JMAXN];
  __shared__ int rotated;
  __shared__ int pairs_left;
  __shared__ int wrot[JNT / 64];  // rotations of the last sweep per wave
  const int b = blockIdx.x, tid = threadIdx.x;
  const int g = tid >> 4, sub = tid & 15;  // 64 groups of 16 lanes
  constexpr int NG = JNT / 16;
  const int ld = n + 1;
  for (int e = tid; e < n * n; e += JNT) {
    const int i = e % n, j = e / n;
    Wl[j * ld + i] = ldv(A, b, i, j);
  }
  __syncthreads();
  int myrot = 0;  // rotations of this lane's pairs in the current sweep
  const int npad = n + (n & 1);
  const int npairs = npad / 2;
  const double tol = 8.0 * 2.220446049250313e-16 * sqrt((double)n);
  for (int sweep = 0; sweep < 40 && n > 1; ++sweep) {
    for (int c = tid; c < n; c += JNT) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += cabs2(Wl[c * ld + i]);
      nrm2[c] = s;
    }
    {
      int cnt = myrot;
      myrot = 0;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
      if ((tid & 63) == 0) wrot[tid >> 6] = cnt;
    }
    if (tid == 0) {
      rotated = 0;
      pairs_left = 0;
    }
    __syncthreads();
    int last_rot = 0;
#pragma unroll
    for (int i = 0; i < JNT / 64; ++i) last_rot += wrot[i];
    // once a sweep rotated at most n^2 / 8 pairs (a quarter of them:
    // convergence is near), all pairs are tested at once before the next: a
    // sweep that would find none to rotate is not run
    if (sweep > 0 && 8 * last_rot <= n * n) {
      if (jac_pairs_left(n, ld, Wl, nrm2, tol)) pairs_left = 1;
      __syncthreads();
      if (!pairs_left) break;
    }
    for (int r = 0; r < npad - 1; ++r) {
      for (int p = g; p < npairs; p += NG) {
        const int pa = p, pb = npad - 1 - p;
        int ca = pa == 0 ? 0 : ((pa - 1 + r) % (npad - 1)) + 1;
        int cb = ((pb - 1 + r) % (npad - 1)) + 1;
        if (ca >= n || cb >= n) continue;
        if (ca > cb) { const int t = ca; ca = cb; cb = t; }
        cplx* xa = Wl + ca * ld;
        cplx* xb = Wl + cb * ld;
        // the pair's rows of this lane in registers: one LDS round trip for
        // the loads, the rotation writes back from them
        constexpr int JR = (JMAXN + 15) / 16;
        cplx va[JR], vb[JR];
#pragma unroll
        for (int q = 0; q < JR; ++q) {
          const int i = min(sub + 16 * q, n - 1);
          va[q] = xa[i];
          vb[q] = xb[i];
        }
        cplx ga = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < JR; ++q) {
          if (sub + 16 * q >= n) continue;
          const cplx t = cdotc(va[q], vb[q]);
          ga = make_double2(ga.x + t.x, ga.y + t.y);
        }
        // the 16 lanes of a pair are one DPP row
        ga.x = row16_sum(ga.x);
        ga.y = row16_sum(ga.y);
        const double al = nrm2[ca], be = nrm2[cb];
        const double gg2 = cabs2(ga);
        if (!(gg2 > tol * tol * (al * be)) || al < 1e-300 || be < 1e-300) continue;
        // rotation angle: t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
        // zeta = (be - al) / (2 |ga|), written as w / (1 + sqrt(1 + w^2)) with
        // w = 1 / |zeta| for |zeta| > 1 so no square overflows; reciprocals and
        // square roots from the hardware estimates with a Newton step (the
        // chain is on the critical path of every rotation round)
        const double rg = rsq_nt(gg2), gg = gg2 * rg;
        const double zeta = (be - al) * (0.5 * rg);
        const double z = fabs(zeta);
        const bool big = z > 1.0;
        const double wz = big ? rcp_nt(z) : z;
        const double s1 = sqrt_nt(fma(wz, wz, 1.0));
        const double ta = big ? wz * rcp_nt(1.0 + s1) : rcp_nt(z + s1);
        const double t = zeta >= 0.0 ? ta : -ta;
        const double cs = rsq_nt(fma(t, t, 1.0)), sn = cs * t;
        const cplx ph = make_double2(ga.x * rg, -ga.y * rg);
#pragma unroll
        for (int q = 0; q < JR; ++q) {
          const int i = sub + 16 * q;
          if (i >= n) continue;
          const cplx u = va[q], wv = cmul(ph, vb[q]);
          xa[i] = make_double2(cs * u.x - sn * wv.x, cs * u.y - sn * wv.y);
          xb[i] = make_double2(sn * u.x + cs * wv.x, sn * u.y + cs * wv.y);
        }
        if (sub == 0) {
          nrm2[ca] = al - t * gg;
          nrm2[cb] = be + t * gg;
          rotated = 1;
          ++myrot;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  for (int c = tid; c < n; c += JNT) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += cabs2(Wl[c * ld + i]);
    sig[c] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < n; j += JNT) {
    const double sj = sig[j];
    int pos = 0;
    for (int i = 0; i < n; ++i) {
      const double si = sig[i];
      pos += (si > sj) || (si == sj && i < j);
    }
    rankpos[j] = pos;
  }
  __syncthreads();
  for (int j = tid; j < n; j += JNT) S[(long)b * n + rankpos[j]] = sig[j];
  for (int e = tid; e < n * n; e += JNT) {
    const int i = e / n, j = e % n;
    const double sj = sig[j];
    cplx u = Wl[j * ld + i];
    if (sj > 0.0) { u.x /= sj; u.y /= sj; }
    else u = make_double2(0.0, 0.0);
    U.base[b * U.sb + (long)i * U.rs + (long)rankpos[j] * U.cs] = u;
  }
}

// The same one-sided Jacobi for 96 < n <= 320, where the square matrix
// (up to 1.6 MB) outgrows the 160 KB of LDS: the first nA columns stay in
// LDS, the others live in a per-matrix workspace slice (global memory,
// L2-resident); a column is addressed through a flat pointer to either, so
// the rotation loop is the LDS kernel's.  LP lanes cooperate on a column
// pair: 16 up to n = 160, 32 beyond (ten rows per lane either way).
constexpr int JBIGN = 320;

__device__ __forceinline__ cplx* jcol(cplx* Wl, cplx* Wg, int nA, int n, int c) {
  return c < nA ? Wl + (long)c * n : Wg + (long)(c - nA) * n;
}

template <int LP>
__global__ __launch_bounds__(JNT) void k_jacobi_hyb(int n, int nA, MatView A, MatOut U, double* S,
                                                    cplx* gws, long gsz) {
  extern __shared__ cplx Wl[];  // columns [0, nA), column-major
  __shared__ double nrm2[JBIGN];
  __shared__ double sig[JBIGN];
  __shared__ int rankpos[JBIGN];
  __shared__ int rotated;
  const int b = blockIdx.x, tid = threadIdx.x;
  const int g = tid / LP, sub = tid % LP;
  constexpr int NG = JNT / LP;
  cplx* Wg = gws + (long)b * gsz;  // columns [nA, n)
  for (int e = tid; e < n * n; e += JNT) {
    const int i = e % n, j = e / n;
    jcol(Wl, Wg, nA, n, j)[i] = ldv(A, b, i, j);
  }
  __syncthreads();
  const int npad = n + (n & 1);
  const int npairs = npad / 2;
  const double tol = 8.0 * 2.220446049250313e-16 * sqrt((double)n);
  for (int sweep = 0; sweep < 40 && n > 1; ++sweep) {
    for (int c = tid; c < n; c += JNT) {
      const cplx* xc = jcol(Wl, Wg, nA, n, c);
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += cabs2(xc[i]);
      nrm2[c] = s;
    }
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < npad - 1; ++r) {
      for (int p = g; p < npairs; p += NG) {
        const int pa = p, pb = npad - 1 - p;
        int ca = pa == 0 ? 0 : ((pa - 1 + r) % (npad - 1)) + 1;
        int cb = ((pb - 1 + r) % (npad - 1)) + 1;
        if (ca >= n || cb >= n) continue;
        if (ca > cb) { const int t = ca; ca = cb; cb = t; }
        cplx* xa = jcol(Wl, Wg, nA, n, ca);
        cplx* xb = jcol(Wl, Wg, nA, n, cb);
        constexpr int JR = 10;  // rows per lane: n <= LP * JR (160 or 320)
        cplx va[JR], vb[JR];
#pragma unroll
        for (int q = 0; q < JR; ++q) {
          const int i = min(sub + LP * q, n - 1);
          va[q] = xa[i];
          vb[q] = xb[i];
        }
        cplx ga = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < JR; ++q) {
          if (sub + LP * q >= n) continue;
          const cplx t = cdotc(va[q], vb[q]);
          ga = make_double2(ga.x + t.x, ga.y + t.y);
        }
        ga.x = row16_sum(ga.x);
        ga.y = row16_sum(ga.y);
        if (LP == 32) {
          ga.x += __shfl_xor(ga.x, 16);
          ga.y += __shfl_xor(ga.y, 16);
        }
        const double al = nrm2[ca], be = nrm2[cb];
        const double gg2 = cabs2(ga);
        if (!(gg2 > tol * tol * (al * be)) || al < 1e-300 || be < 1e-300) continue;
        const double rg = rsq_nt(gg2), gg = gg2 * rg;
        const double zeta = (be - al) * (0.5 * rg);
        const double z = fabs(zeta);
        const bool big = z > 1.0;
        const double wz = big ? rcp_nt(z) : z;
        const double s1 = sqrt_nt(fma(wz, wz, 1.0));
        const double ta = big ? wz * rcp_nt(1.0 + s1) : rcp_nt(z + s1);
        const double t = zeta >= 0.0 ? ta : -ta;
        const double cs = rsq_nt(fma(t, t, 1.0)), sn = cs * t;
        const cplx ph = make_double2(ga.x * rg, -ga.y * rg);
#pragma unroll
        for (int q = 0; q < JR; ++q) {
          const int i = sub + LP * q;
          if (i >= n) continue;
          const cplx u = va[q], wv = cmul(ph, vb[q]);
          xa[i] = make_double2(cs * u.x - sn * wv.x, cs * u.y - sn * wv.y);
          xb[i] = make_double2(sn * u.x + cs * wv.x, sn * u.y + cs * wv.y);
        }
        if (sub == 0) {
          nrm2[ca] = al - t * gg;
          nrm2[cb] = be + t * gg;
          rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  for (int c = tid; c < n; c += JNT) {
    const cplx* xc = jcol(Wl, Wg, nA, n, c);
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += cabs2(xc[i]);
    sig[c] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < n; j += JNT) {
    const double sj = sig[j];
    int pos = 0;
    for (int i = 0; i < n; ++i) {
      const double si = sig[i];
      pos += (si > sj) || (si == sj && i < j);
    }
    rankpos[j] = pos;
  }
  __syncthreads();
  for (int j = tid; j < n; j += JNT) S[(long)b * n + rankpos[j]] = sig[j];
  for (int e = tid; e < n * n; e += JNT) {
    const int i = e / n, j = e % n;
    const double sj = sig[j];
    cplx u = jcol(Wl, Wg, nA, n, j)[i];
    if (sj > 0.0) { u.x /= sj; u.y /= sj; }
    else u = make_double2(0.0, 0.0);
    U.base[b * U.sb + (long)i * U.rs + (long)rankpos[j] * U.cs] = u;
  }
}

// columns of an n x n Jacobi matrix that stay in LDS (the rest go to the
// workspace): as many as 150 KB of dynamic LDS hold (the static arrays of
// n = 320 take another 6.4 KB of the 160 KB)
static int jacobi_lds_cols(int n) {
  const int c = (int)((150L * 1024) / (16L * n));
  return c < n ? c : n;
}

}  // namespace

size_t qr_fast_ws(int batch, int m, int n) {
  const long k = m < n ? m : n;
  return (size_t)batch * ((size_t)m * k + k);
}

template <int RB, int CG>
bool qr2d_any(int batch, int m, int n, const MatView& A, const MatOut& R, const MatOut& Q, hipStream_t s,
              cplx* vout = nullptr, const int* only = nullptr) {
  return try_qr_2d<RB, 4, CG>(batch, m, n, A, R, Q, s, vout, only) ||
         try_qr_2d<RB, 8, CG>(batch, m, n, A, R, Q, s, vout, only) ||
         try_qr_2d<RB, 12, CG>(batch, m, n, A, R, Q, s, vout, only) ||
         try_qr_2d<RB, 14, CG>(batch, m, n, A, R, Q, s, vout, only);
}

bool qr_one_rowblock(int batch, int m, int n, const MatView& A, const MatOut& R, cplx* vout,
                     hipStream_t s) {
  return qr_1r_dispatch(batch, m, n, A, R, vout, s);
}

bool qr_2d_vectors(int batch, int m, int n, MatView A, MatOut R, cplx* ws, hipStream_t s, const int* only) {
  // one wave per column group wins only for short columns (24 x 24: 42 us
  // against 59 us; 160 x 80: 373 us against 189 us for R)
  if (only == nullptr && m <= 32 && qr_one_rowblock(batch, m, n, A, R, ws, s)) return true;
  const MatOut Q{nullptr, 0, 0, 0};
  switch ((n + 15) / 16) {
    case 2: return qr2d_any<8, 2>(batch, m, n, A, R, Q, s, ws, only);
    case 3: return qr2d_any<5, 3>(batch, m, n, A, R, Q, s, ws, only);
    case 4: return qr2d_any<4, 4>(batch, m, n, A, R, Q, s, ws, only);
    case 5: return qr2d_any<3, 5>(batch, m, n, A, R, Q, s, ws, only);
    case 6: return qr2d_any<2, 6>(batch, m, n, A, R, Q, s, ws, only);
    default: return false;
  }
}

bool qr_fast(int batch, int m, int n, MatView A, MatOut R, MatOut Q, cplx* ws, hipStream_t s) {
  if (batch <= 0 || m <= 0 || n <= 0) return true;
  // 2D wave grid: RB row blocks x CG groups of 16 columns (<= 16 waves);
  // variants that would spill registers are left out
  bool done = false;
  switch ((n + 15) / 16) {
    case 1: done = qr2d_any<8, 1>(batch, m, n, A, R, Q, s) || try_qr_2d<8, 16, 1>(batch, m, n, A, R, Q, s); break;
    case 2: done = qr2d_any<8, 2>(batch, m, n, A, R, Q, s); break;
    case 3: done = qr2d_any<5, 3>(batch, m, n, A, R, Q, s); break;
    case 4: done = qr2d_any<4, 4>(batch, m, n, A, R, Q, s); break;
    case 5: done = qr2d_any<3, 5>(batch, m, n, A, R, Q, s); break;
    case 6: done = qr2d_any<2, 6>(batch, m, n, A, R, Q, s) || try_qr_2d<2, 16, 6>(batch, m, n, A, R, Q, s); break;
    case 7: done = qr2d_any<2, 7>(batch, m, n, A, R, Q, s); break;
    case 8: done = qr2d_any<2, 8>(batch, m, n, A, R, Q, s); break;
    default: break;
  }
  if (done) return true;
  if (n <= 64) {
    if (try_qr_lc<8, 16, 1>(batch, m, n, A, R, Q, s) || try_qr_lc<8, 24, 1>(batch, m, n, A, R, Q, s) ||
        try_qr_lc<8, 32, 1>(batch, m, n, A, R, Q, s))
      return true;
    return try_qr_rows<4, 8>(batch, m, n, A, R, Q, ws, s);
  }
  if (try_qr_lc<8, 16, 2>(batch, m, n, A, R, Q, s) || try_qr_lc<16, 10, 2>(batch, m, n, A, R, Q, s))
    return true;
  return try_qr_rows<2, 16>(batch, m, n, A, R, Q, ws, s) || try_qr_rows<3, 16>(batch, m, n, A, R, Q, ws, s);
}

bool qr_two_col(int batch, int m, int n, MatView A, MatOut R, MatOut Q, hipStream_t s) {
  if (batch <= 0 || m <= 0 || n <= 0) return true;
  switch ((n + 31) / 32) {
    case 1: return try_qr_2c<8, 4, 1, 2>(batch, m, n, A, R, Q, s) || try_qr_2c<8, 8, 1, 2>(batch, m, n, A, R, Q, s);
    case 2: return try_qr_2c<8, 4, 2, 2>(batch, m, n, A, R, Q, s) || try_qr_2c<8, 8, 2, 2>(batch, m, n, A, R, Q, s);
    case 3: return try_qr_2c<5, 4, 3, 2>(batch, m, n, A, R, Q, s) || try_qr_2c<5, 8, 3, 2>(batch, m, n, A, R, Q, s) ||
                   try_qr_2c<5, 12, 3, 2>(batch, m, n, A, R, Q, s);
    default: return false;
  }
}

size_t jacobi_ws(int batch, int n) {
  if (n <= JMAXN) return 0;
  return (size_t)batch * (size_t)(n - jacobi_lds_cols(n)) * n;
}

bool jacobi_big(int batch, int n, MatView A, MatOut U, double* S, cplx* ws, hipStream_t s) {
  if (batch <= 0 || n <= 0) return true;
  if (n <= JMAXN || n > JBIGN || ws == nullptr) return false;
  static const bool attr = [&]() {
    check(hipFuncSetAttribute((const void*)k_jacobi_hyb<16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              150 * 1024),
          "jacobi_hyb lds attribute");
    check(hipFuncSetAttribute((const void*)k_jacobi_hyb<32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              150 * 1024),
          "jacobi_hyb lds attribute");
    return true;
  }();
  (void)attr;
  const int nA = jacobi_lds_cols(n);
  const size_t shm = (size_t)nA * n * sizeof(cplx);
  if (n <= 160)
    hipLaunchKernelGGL(k_jacobi_hyb<16>, dim3(batch), dim3(JNT), shm, s, n, nA, A, U, S, ws,
                       (long)(n - nA) * n);
  else
    hipLaunchKernelGGL(k_jacobi_hyb<32>, dim3(batch), dim3(JNT), shm, s, n, nA, A, U, S, ws,
                       (long)(n - nA) * n);
  check(hipGetLastError(), "jacobi_hyb launch");
  return true;
}

bool jacobi_square(int batch, int n, MatView A, MatOut U, double* S, hipStream_t s) {
  if (batch <= 0 || n <= 0) return true;
  if (n > JMAXN) return false;
  // once per kernel and process (thread-safe static initialisation: the
  // load-case groups of a solve launch from several host threads)
  static const bool attr = [&]() {
    check(hipFuncSetAttribute((const void*)k_jacobi_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                              JMAXN * (JMAXN + 1) * (int)sizeof(cplx)),
          "jacobi lds attribute");
    return true;
  }();
  (void)attr;
  const size_t shm = (size_t)n * (n + 1) * sizeof(cplx);
  hipLaunchKernelGGL(k_jacobi_lds, dim3(batch), dim3(JNT), shm, s, n, A, U, S);
  check(hipGetLastError(), "jacobi_lds launch");
  return true;
}

}  // namespace qtt
