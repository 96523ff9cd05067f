// HIP kernels for quantized tensor-train arithmetic on gfx950 (CDNA4).
//
// Everything here works on interleaved complex FP64 (double2) data:
//  * a strided, two-level batched complex GEMM (LDS-tiled) that carries the
//    core-by-core contractions of TTO x TT products, sketches and absorbs;
//  * Householder QR with 64-lane wavefront-shuffle reductions for the norms
//    and reflector dot products (orthogonalisation sweeps of TT-rounding,
//    Sec. 3 of the paper);
//  * one-sided Jacobi SVD (truncation sweeps of TT-rounding), singular
//    values sorted on device;
//  * Philox4x32-10 + Box-Muller complex normals for the rounding sketches;
//  * the materialised TTO x TT core product (Table 2, contract), a purely
//    HBM-bound kernel with coalesced rank-major writes.
#include "qtt_internal.h"

#include <cstdio>
#include <stdexcept>

namespace qtt {

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    throw std::runtime_error(std::string("HIP error in ") + what + ": " +
                             hipGetErrorString(e));
  }
}

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ cplx cconj(cplx a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ cplx csub(cplx a, cplx b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
// conj(a) * b
__device__ __forceinline__ cplx cdotc(cplx a, cplx b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double cabs2(cplx a) { return a.x * a.x + a.y * a.y; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ cplx wave_sum(cplx v) {
  return make_double2(wave_sum(v.x), wave_sum(v.y));
}

// Block-wide sum of a double; every thread gets the result.
template <int NT>
__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += sh[i];
  return t;
}

__device__ __forceinline__ cplx ldview(const MatView& v, long b, long i, long j) {
  cplx a = v.base[b * v.sb + i * v.rs + j * v.cs];
  if (v.conj) a.y = -a.y;
  return a;
}

// ---------------------------------------------------------------------------
// GEMM
// ---------------------------------------------------------------------------
constexpr int GBK = 8;

template <int TM, int TN>
__global__ __launch_bounds__((TM / 4) * (TN / 4)) void k_gemm(GemmArgs g) {
  constexpr int NT = (TM / 4) * (TN / 4);
  constexpr int TX = TN / 4;  // threads along N
  __shared__ cplx As[GBK][TM];
  __shared__ cplx Bs[GBK][TN];
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  long oa, ob, oc;
  gemm_batch_offsets(g, blockIdx.z, oa, ob, oc);
  const cplx* A = g.A + oa;
  const cplx* B = g.B + ob;
  cplx* C = g.C + oc;

  cplx acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);

  for (int k0 = 0; k0 < g.K; k0 += GBK) {
    for (int e = tid; e < TM * GBK; e += NT) {
      int mm, kk;
      if (g.opA == OP_N) { kk = e % GBK; mm = e / GBK; }
      else { mm = e % TM; kk = e / TM; }
      const int m = m0 + mm, k = k0 + kk;
      cplx v = make_double2(0.0, 0.0);
      if (m < g.M && k < g.K) {
        if (g.opA == OP_N) v = A[(long)m * g.lda + k];
        else {
          v = A[(long)k * g.lda + m];
          if (g.opA == OP_C) v.y = -v.y;
        }
      }
      As[kk][mm] = v;
    }
    for (int e = tid; e < TN * GBK; e += NT) {
      int nn, kk;
      if (g.opB == OP_N) { nn = e % TN; kk = e / TN; }
      else { kk = e % GBK; nn = e / GBK; }
      const int n = n0 + nn, k = k0 + kk;
      cplx v = make_double2(0.0, 0.0);
      if (n < g.N && k < g.K) {
        if (g.opB == OP_N) v = B[(long)k * g.ldb + n];
        else {
          v = B[(long)n * g.ldb + k];
          if (g.opB == OP_C) v.y = -v.y;
        }
      }
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GBK; ++kk) {
      cplx a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + i * (TM / 4)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + j * TX];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j].x = fma(a[i].x, b[j].x, acc[i][j].x);
          acc[i][j].x = fma(-a[i].y, b[j].y, acc[i][j].x);
          acc[i][j].y = fma(a[i].x, b[j].y, acc[i][j].y);
          acc[i][j].y = fma(a[i].y, b[j].x, acc[i][j].y);
        }
    }
    __syncthreads();
  }
  const bool zb = (g.beta.x == 0.0 && g.beta.y == 0.0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty + i * (TM / 4);
    if (m >= g.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx + j * TX;
      if (n >= g.N) continue;
      cplx r = cmul(g.alpha, acc[i][j]);
      cplx* cp = C + (long)m * g.ldc + n;
      if (!zb) r = cadd(r, cmul(g.beta, *cp));
      *cp = r;
    }
  }
}

template <int TM, int TN>
static void launch_gemm(const GemmArgs& g, hipStream_t s) {
  dim3 grid((g.N + TN - 1) / TN, (g.M + TM - 1) / TM, (unsigned)gemm_nbatch(g));
  hipLaunchKernelGGL((k_gemm<TM, TN>), grid, dim3((TM / 4) * (TN / 4)), 0, s, g);
}

bool gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.nb1 <= 0 || g.nb2 <= 0 || g.nb3 <= 0) return false;
  if (gemm_nbatch(g) > 65535) throw std::runtime_error("gemm: batch too large");
  if (gemm_mfma(g, s)) return true;
  gemm_vector(g, s);
  return false;
}

void gemm_vector(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.nb1 <= 0 || g.nb2 <= 0 || g.nb3 <= 0) return;
  if (gemm_nbatch(g) > 65535) throw std::runtime_error("gemm: batch too large");
  const long tiles64 = (long)((g.M + 63) / 64) * ((g.N + 63) / 64) * gemm_nbatch(g);
  if (g.M <= 16 && g.N > 32) launch_gemm<16, 64>(g, s);
  else if (g.N <= 16 && g.M > 32) launch_gemm<64, 16>(g, s);
  else if (g.M <= 32 || g.N <= 32 || tiles64 < 512) launch_gemm<32, 32>(g, s);
  else launch_gemm<64, 64>(g, s);
  check(hipGetLastError(), "gemm launch");
}

// ---------------------------------------------------------------------------
// Householder QR (one workgroup per matrix)
// ---------------------------------------------------------------------------
constexpr int QR_NT = 512;

__global__ __launch_bounds__(QR_NT) void k_qr(int m, int n, MatView A, MatOut R,
                                              MatOut Q, cplx* ws) {
  const int b = blockIdx.x;
  const int k = min(m, n);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = QR_NT / 64;
  cplx* W = ws + (long)b * ((long)m * n + (long)m * k + k);
  cplx* Qw = W + (long)m * n;
  cplx* tau = Qw + (long)m * k;
  __shared__ double red[NW];
  __shared__ cplx sh_tau, sh_inv;

  for (long e = tid; e < (long)m * n; e += QR_NT) {
    const long i = e % m, j = e / m;
    W[j * m + i] = ldview(A, b, i, j);
  }
  __syncthreads();

  for (int j = 0; j < k; ++j) {
    cplx* v = W + (long)j * m;
    double part = 0.0;
    for (int i = j + 1 + tid; i < m; i += QR_NT) part += cabs2(v[i]);
    const double xn2 = block_sum<QR_NT>(part, red);
    if (tid == 0) {
      const cplx alpha = v[j];
      if ((xn2 == 0.0 && alpha.y == 0.0) || cabs2(alpha) + xn2 < QR_TINY) {
        sh_tau = make_double2(0.0, 0.0);
        sh_inv = make_double2(0.0, 0.0);
      } else {
        const double beta = -copysign(sqrt(cabs2(alpha) + xn2), alpha.x);
        sh_tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        const cplx d = make_double2(alpha.x - beta, alpha.y);
        const double dd = cabs2(d);
        sh_inv = make_double2(d.x / dd, -d.y / dd);
        v[j] = make_double2(beta, 0.0);
      }
      tau[j] = sh_tau;
    }
    __syncthreads();
    const cplx tj = sh_tau;
    if (tj.x == 0.0 && tj.y == 0.0) continue;
    const cplx inv = sh_inv;
    for (int i = j + 1 + tid; i < m; i += QR_NT) v[i] = cmul(v[i], inv);
    __syncthreads();
    const cplx ctj = cconj(tj);
    for (int c = j + 1 + wave; c < n; c += NW) {
      cplx* col = W + (long)c * m;
      cplx s = (lane == 0) ? col[j] : make_double2(0.0, 0.0);
      for (int i = j + 1 + lane; i < m; i += 64) s = cadd(s, cdotc(v[i], col[i]));
      s = wave_sum(s);
      const cplx f = cmul(ctj, s);
      if (lane == 0) col[j] = csub(col[j], f);
      for (int i = j + 1 + lane; i < m; i += 64) col[i] = csub(col[i], cmul(f, v[i]));
    }
    __syncthreads();
  }

  for (long e = tid; e < (long)k * n; e += QR_NT) {
    const long i = e / n, j = e % n;
    const cplx val = (i <= j) ? W[j * m + i] : make_double2(0.0, 0.0);
    R.base[b * R.sb + i * R.rs + j * R.cs] = val;
  }
  if (Q.base == nullptr) return;

  for (long e = tid; e < (long)m * k; e += QR_NT) {
    const long i = e % m, j = e / m;
    Qw[j * m + i] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    const cplx tj = tau[j];
    if (tj.x == 0.0 && tj.y == 0.0) continue;
    const cplx* v = W + (long)j * m;
    for (int c = j + wave; c < k; c += NW) {
      cplx* col = Qw + (long)c * m;
      cplx s = (lane == 0) ? col[j] : make_double2(0.0, 0.0);
      for (int i = j + 1 + lane; i < m; i += 64) s = cadd(s, cdotc(v[i], col[i]));
      s = wave_sum(s);
      const cplx f = cmul(tj, s);
      if (lane == 0) col[j] = csub(col[j], f);
      for (int i = j + 1 + lane; i < m; i += 64) col[i] = csub(col[i], cmul(f, v[i]));
    }
    __syncthreads();
  }
  for (long e = tid; e < (long)m * k; e += QR_NT) {
    const long i = e / k, j = e % k;
    Q.base[b * Q.sb + i * Q.rs + j * Q.cs] = Qw[j * m + i];
  }
}

size_t qr_ws(int batch, int m, int n) {
  return (size_t)batch * qr_ws_per_matrix(m, n);
}

void qr(int batch, int m, int n, MatView A, MatOut R, MatOut Q, cplx* ws,
        hipStream_t s) {
  if (batch <= 0 || m <= 0 || n <= 0) return;
  // beyond what one compute unit holds (more than 192 rows or 96 columns):
  // the workspace-resident blocked kernel (288 x 144 with Q: 5.2 ms in the
  // global-memory kernel)
  if ((m > 192 || n > 96) && qr_big(batch, m, n, A, R, Q, ws, s)) return;
  // the blocked matrix-core kernel beats the unblocked register kernels
  // only beyond 80 columns (192 x 96: 0.72 ms against 1.46 ms with Q;
  // 160 x 80: 0.52 ms against 0.39 ms)
  if (n > 80 && qr_blocked(batch, m, n, A, R, Q, ws, s)) return;
  // R from the unblocked register kernel, Q from its Householder vectors
  // as block reflectors on the matrix cores (160 x 80: Q formation 70 us
  // against 157 us in the register kernel)
  if (m >= n && n > 16 && n <= 96 && m <= 192) {
    if (Q.base != nullptr) {
      if (qr_2d_vectors(batch, m, n, A, R, ws, s)) {
        if (!qr_form_q(batch, m, n, Q, ws, s)) throw std::logic_error("qr: Q formation shape");
        return;
      }
    } else if (m <= 32 && qr_one_rowblock(batch, m, n, A, R, nullptr, s)) {
      return;
    }
  }
  if (qr_fast(batch, m, n, A, R, Q, ws, s)) return;
  qr_generic(batch, m, n, A, R, Q, ws, s);
}

void qr_generic(int batch, int m, int n, MatView A, MatOut R, MatOut Q, cplx* ws,
                hipStream_t s) {
  if (batch <= 0 || m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_qr, dim3(batch), dim3(QR_NT), 0, s, m, n, A, R, Q, ws);
  check(hipGetLastError(), "qr launch");
}

// ---------------------------------------------------------------------------
// One-sided Jacobi SVD (one workgroup per matrix), m >= n
// ---------------------------------------------------------------------------
constexpr int SVD_NT = 512;
constexpr int SVD_MAXN = 1024;

__global__ __launch_bounds__(SVD_NT) void k_svd(int m, int n, MatView A, MatOut U,
                                                double* S, MatOut V, cplx* ws) {
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = SVD_NT / 64;
  cplx* W = ws + (long)b * ((long)m * n + (long)n * n);
  cplx* Vw = W + (long)m * n;
  __shared__ double sig[SVD_MAXN];
  __shared__ int rankpos[SVD_MAXN];
  __shared__ int rotated;

  for (long e = tid; e < (long)m * n; e += SVD_NT) {
    const long i = e % m, j = e / m;
    W[j * m + i] = ldview(A, b, i, j);
  }
  for (long e = tid; e < (long)n * n; e += SVD_NT) {
    const long i = e % n, j = e / n;
    Vw[j * n + i] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();

  const int npad = n + (n & 1);
  const int npairs = npad / 2;
  const double tol = 8.0 * 2.220446049250313e-16 * sqrt((double)m);
  for (int sweep = 0; sweep < 40 && n > 1; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < npad - 1; ++r) {
      for (int p = wave; p < npairs; p += NW) {
        const int pa = p, pb = npad - 1 - p;
        int ca = pa == 0 ? 0 : ((pa - 1 + r) % (npad - 1)) + 1;
        int cb = ((pb - 1 + r) % (npad - 1)) + 1;
        if (ca >= n || cb >= n) continue;
        if (ca > cb) { const int t = ca; ca = cb; cb = t; }
        cplx* xa = W + (long)ca * m;
        cplx* xb = W + (long)cb * m;
        double al = 0.0, be = 0.0;
        cplx ga = make_double2(0.0, 0.0);
        for (int i = lane; i < m; i += 64) {
          const cplx u = xa[i], w = xb[i];
          al += cabs2(u);
          be += cabs2(w);
          ga = cadd(ga, cdotc(u, w));
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        const double g = sqrt(cabs2(ga));
        if (!(g > tol * sqrt(al * be)) || al < 1e-300 || be < 1e-300) continue;
        if (lane == 0) rotated = 1;
        const double zeta = (be - al) / (2.0 * g);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
        const cplx ph = make_double2(ga.x / g, -ga.y / g);  // e^{-i phi}
        for (int i = lane; i < m; i += 64) {
          const cplx u = xa[i], w = cmul(ph, xb[i]);
          xa[i] = make_double2(c * u.x - sn * w.x, c * u.y - sn * w.y);
          xb[i] = make_double2(sn * u.x + c * w.x, sn * u.y + c * w.y);
        }
        cplx* va = Vw + (long)ca * n;
        cplx* vb = Vw + (long)cb * n;
        for (int i = lane; i < n; i += 64) {
          const cplx u = va[i], w = cmul(ph, vb[i]);
          va[i] = make_double2(c * u.x - sn * w.x, c * u.y - sn * w.y);
          vb[i] = make_double2(sn * u.x + c * w.x, sn * u.y + c * w.y);
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }

  for (int j = wave; j < n; j += NW) {
    const cplx* x = W + (long)j * m;
    double s2 = 0.0;
    for (int i = lane; i < m; i += 64) s2 += cabs2(x[i]);
    s2 = wave_sum(s2);
    if (lane == 0) sig[j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = tid; j < n; j += SVD_NT) {
    const double sj = sig[j];
    int pos = 0;
    for (int i = 0; i < n; ++i) {
      const double si = sig[i];
      pos += (si > sj) || (si == sj && i < j);
    }
    rankpos[j] = pos;
  }
  __syncthreads();
  for (int j = tid; j < n; j += SVD_NT) S[(long)b * n + rankpos[j]] = sig[j];
  for (long e = tid; e < (long)m * n; e += SVD_NT) {
    const long i = e / n, j = e % n;
    const double sj = sig[j];
    cplx u = W[j * m + i];
    if (sj > 0.0) { u.x /= sj; u.y /= sj; }
    else u = make_double2(0.0, 0.0);
    U.base[b * U.sb + i * U.rs + (long)rankpos[j] * U.cs] = u;
  }
  for (long e = tid; e < (long)n * n; e += SVD_NT) {
    const long i = e / n, j = e % n;
    V.base[b * V.sb + i * V.rs + (long)rankpos[j] * V.cs] = Vw[j * n + i];
  }
}

size_t svd_ws(int batch, int m, int n) {
  return (size_t)batch * ((size_t)m * n + (size_t)n * n);
}

void svd(int batch, int m, int n, MatView A, MatOut U, double* S, MatOut V,
         cplx* ws, hipStream_t s) {
  if (batch <= 0 || n <= 0) return;
  if (m < n) throw std::runtime_error("svd: needs m >= n");
  if (n > SVD_MAXN) throw std::runtime_error("svd: n too large");
  hipLaunchKernelGGL(k_svd, dim3(batch), dim3(SVD_NT), 0, s, m, n, A, U, S, V, ws);
  check(hipGetLastError(), "svd launch");
}

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw 2011)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                             uint32_t& c3, uint32_t k0, uint32_t k1) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
  const uint32_t h0 = (uint32_t)(p0 >> 32), l0 = (uint32_t)p0;
  const uint32_t h1 = (uint32_t)(p1 >> 32), l1 = (uint32_t)p1;
  const uint32_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
  c0 = n0; c1 = l1; c2 = n2; c3 = l0;
}

// entry e of the complex standard normal stream (seed, stream), scaled:
// Philox4x32-10 on the counter (e, stream), then Box-Muller
__device__ __forceinline__ cplx gaussian_entry(uint64_t e, uint64_t seed, uint64_t stream,
                                               double scale) {
  uint32_t c0 = (uint32_t)e, c1 = (uint32_t)(e >> 32);
  uint32_t c2 = (uint32_t)stream, c3 = (uint32_t)(stream >> 32);
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    philox_round(c0, c1, c2, c3, k0, k1);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  const double u1 = ((double)c0 + 0.5) * 2.3283064365386963e-10;  // (0, 1)
  const double u2 = ((double)c1 + 0.5) * 2.3283064365386963e-10;
  const double rr = sqrt(-2.0 * log(u1)) * scale;
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);
  return make_double2(rr * cs, rr * sn);
}

// every block of a GaussBlocks set in one launch: thread e finds its block
// by the prefix offsets (at most GAUSS_MULTI_MAX compares)
__global__ void k_gaussian_multi(GaussBlocks g, uint64_t seed) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.start[g.n]) return;
  int i = 0;
  while (i + 1 < g.n && e >= g.start[i + 1]) ++i;
  const long el = e - g.start[i];
  g.out[i][el] = gaussian_entry((uint64_t)el, seed, g.stream[i], g.scale[i]);
}

void gaussian_multi(const GaussBlocks& g, uint64_t seed, hipStream_t s) {
  if (g.n <= 0 || g.start[g.n] == 0) return;
  const int nt = 256;
  const long total = g.start[g.n];
  hipLaunchKernelGGL(k_gaussian_multi, dim3((unsigned)((total + nt - 1) / nt)), dim3(nt), 0, s, g, seed);
  check(hipGetLastError(), "gaussian multi launch");
}

// ---------------------------------------------------------------------------
// Materialised TTO x TT core product (Table 2, contract)
// ---------------------------------------------------------------------------
// All cores of a materialised TTO x TT product in one launch.  Block ranges
// are assigned to cores by the descriptors' start_block prefix.  A thread
// owns one (i, column (b, a, c, c2)) of its core's output: it loads its x
// entries once and writes the rho2 outputs a2 of that row segment, so x is
// read once per rho2 outputs instead of once per output, and the
// operator entries, the same for every lane of a wave with one (a), are
// broadcast loads.  Consecutive lanes hold consecutive c2: every store
// instruction writes consecutive output entries.  32-bit offsets inside a
// core (the host checks every core has < 2^31 entries); the column index
// is split by the descriptors' multiply-high dividers.
constexpr int TTO_NT = 256;

__global__ __launch_bounds__(TTO_NT) void k_tto_apply_all(int ncores, const TtoDesc* __restrict__ D) {
  int kc = 0;
  for (int q = 1; q < ncores; ++q)
    if ((long)blockIdx.x >= D[q].start_block) kc = q;
  const TtoDesc d = D[kc];
  const uint32_t dout = (uint32_t)d.dout, rho2 = (uint32_t)d.rho2, r2 = (uint32_t)d.r2;
  const uint32_t cols = (uint32_t)(d.total / (dout * rho2));
  const uint32_t g = (uint32_t)((long)blockIdx.x - d.start_block) * TTO_NT + threadIdx.x;
  if (g >= cols * dout) return;
  const uint32_t i = fdiv(g, d.f_cols), col = g - i * cols;
  const uint32_t t1 = fdiv(col, d.f_r2), c2 = col - t1 * r2;
  const uint32_t t2 = fdiv(t1, d.f_r), c = t1 - t2 * (uint32_t)d.r;
  const uint32_t b = fdiv(t2, d.f_rho), a = t2 - b * (uint32_t)d.rho;
  const uint32_t dx = d.din > 0 ? (uint32_t)d.din : dout;
  const cplx* xb = d.x + ((b * (uint32_t)d.r + c) * dx * r2 + c2);
  const cplx* Ab = d.A + (long)fdiv(b, d.f_group) * d.a_stride;
  cplx* Zb = d.Z + (((t2 * (uint32_t)d.r + c) * dout + i) * rho2 * r2 + c2);
  if (d.din == 0) {
    const cplx xi = xb[i * r2];
    const cplx* Ai = Ab + (a * dout + i) * rho2;
    for (uint32_t a2 = 0; a2 < rho2; ++a2) Zb[a2 * r2] = cmul(Ai[a2], xi);
  } else if (d.din == 2) {
    const cplx x0 = xb[0], x1 = xb[r2];
    const cplx* A0 = Ab + ((a * 2u) * dout + i) * rho2;
    const cplx* A1 = Ab + ((a * 2u + 1u) * dout + i) * rho2;
    for (uint32_t a2 = 0; a2 < rho2; ++a2) Zb[a2 * r2] = cadd(cmul(A0[a2], x0), cmul(A1[a2], x1));
  } else {
    const uint32_t din = (uint32_t)d.din;
    for (uint32_t a2 = 0; a2 < rho2; ++a2) {
      cplx acc = make_double2(0.0, 0.0);
      for (uint32_t j = 0; j < din; ++j)
        acc = cadd(acc, cmul(Ab[((a * din + j) * dout + i) * rho2 + a2], xb[j * r2]));
      Zb[a2 * r2] = acc;
    }
  }
}

long tto_apply_blocks(long total, int rho2) {
  const long threads = total / rho2;  // one per (i, column)
  return (threads + TTO_NT - 1) / TTO_NT;
}

void tto_apply_all(int ncores, const TtoDesc* D_dev, long nblocks, hipStream_t s) {
  if (ncores <= 0 || nblocks <= 0) return;
  if (nblocks > 2147483647L) throw std::runtime_error("tto_apply_all: grid too large");
  hipLaunchKernelGGL(k_tto_apply_all, dim3((unsigned)nblocks), dim3(TTO_NT), 0, s, ncores, D_dev);
  check(hipGetLastError(), "tto_apply_all launch");
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_batch_norm(long len, long stride, const cplx* x,
                                                    double* out) {
  __shared__ double red[4];
  const cplx* p = x + (long)blockIdx.x * stride;
  double s = 0.0;
  for (long e = threadIdx.x; e < len; e += 256) s += cabs2(p[e]);
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(s);
}

void batch_norm(int batch, long len, long stride, const cplx* x, double* out,
                hipStream_t s) {
  if (batch <= 0) return;
  hipLaunchKernelGGL(k_batch_norm, dim3(batch), dim3(256), 0, s, len, stride, x, out);
  check(hipGetLastError(), "batch_norm launch");
}

__global__ void k_scale_cols(long total, int rows, int cols, long ld, long sb, cplx* x,
                             const double* S, long sS) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int j = e % cols;
  const long t = e / cols;
  const int i = t % rows;
  const long b = t / rows;
  cplx* p = x + b * sb + i * ld + j;
  const double w = S[b * sS + j];
  *p = make_double2(p->x * w, p->y * w);
}

void scale_cols(int batch, int rows, int cols, long ld, long sb, cplx* x, const double* S,
                long sS, hipStream_t s) {
  const long total = (long)batch * rows * cols;
  if (total == 0) return;
  hipLaunchKernelGGL(k_scale_cols, dim3((total + 255) / 256), dim3(256), 0, s, total, rows,
                     cols, ld, sb, x, S, sS);
  check(hipGetLastError(), "scale_cols launch");
}

__global__ void k_copy2d(long total, int rows, int cols, MatView in, MatOut out, cplx alpha,
                         const double* bscale) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int j = e % cols;
  const long t = e / cols;
  const int i = t % rows;
  const long b = t / rows;
  cplx a = alpha;
  if (bscale) {
    a.x *= bscale[b];
    a.y *= bscale[b];
  }
  out.base[b * out.sb + i * out.rs + (long)j * out.cs] = cmul(a, ldview(in, b, i, j));
}

void copy2d(int batch, int rows, int cols, MatView in, MatOut out, cplx alpha,
            hipStream_t s, const double* bscale) {
  const long total = (long)batch * rows * cols;
  if (total == 0) return;
  hipLaunchKernelGGL(k_copy2d, dim3((total + 255) / 256), dim3(256), 0, s, total, rows, cols,
                     in, out, alpha, bscale);
  check(hipGetLastError(), "copy2d launch");
}

void conj_transpose(int batch, int rows, int keep, MatView in, MatOut out, hipStream_t s) {
  // out(j, i) = conj(in(i, j)) for j < keep
  MatView t = in;
  t.conj = !in.conj;
  std::swap(t.rs, t.cs);
  copy2d(batch, keep, rows, t, out, make_double2(1.0, 0.0), s);
}

__global__ void k_span_arm(unsigned long long* t, int slots) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < slots) {
    t[2 * i] = ~0ull;
    t[2 * i + 1] = 0ull;
  }
}

void span_arm(unsigned long long* t, int slots, hipStream_t s) {
  if (slots <= 0) return;
  hipLaunchKernelGGL(k_span_arm, dim3((slots + 255) / 256), dim3(256), 0, s, t, slots);
  check(hipGetLastError(), "span arm launch");
}

__global__ void k_fill(cplx* p, size_t count, cplx v) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = v;
}

void fill(cplx* p, size_t count, cplx v, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_fill, dim3((count + 255) / 256), dim3(256), 0, s, p, count, v);
  check(hipGetLastError(), "fill launch");
}

// One-hot expansion of a voxel phase array: out[p * NN + v] = 1 if
// phase[v] == p else 0, p < nphase; *bad is set when a phase id is out of
// range.
__global__ void k_onehot(const uint8_t* __restrict__ phase, long NN, int nphase, cplx* __restrict__ out,
                         int* bad) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= NN) return;
  const int ph = phase[v];
  if (ph >= nphase) *bad = 1;
  for (int p = 0; p < nphase; ++p) out[(long)p * NN + v] = make_double2(ph == p ? 1.0 : 0.0, 0.0);
}

void onehot(const uint8_t* phase, long NN, int nphase, cplx* out, int* bad, hipStream_t s) {
  if (NN <= 0) return;
  hipLaunchKernelGGL(k_onehot, dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, s, phase, NN, nphase,
                     out, bad);
  check(hipGetLastError(), "onehot launch");
}

// Unit momentum directions of the Green factors: out[c * NN + e], e =
// (x N + y) N + z, c = (sigma, a) with a < 3: f_a / |f| for f = (f[x],
// f[y], f[z]) (sigma = 0) and the same with the other Nyquist
// representative f2 (sigma = 1, same |f|); 0 at the zero frequency.  f and
// f2 hold one axis's momentum frequencies.
__global__ void k_direction(const double* __restrict__ f, const double* __restrict__ f2, int n, long NN,
                            cplx* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NN) return;
  const int N = 1 << n;
  const int x = (int)(e >> (2 * n)), y = (int)((e >> n) & (N - 1)), z = (int)(e & (N - 1));
  const double r2 = f[x] * f[x] + f[y] * f[y] + f[z] * f[z];
  const double inv = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
  out[0 * NN + e] = make_double2(f[x] * inv, 0.0);
  out[1 * NN + e] = make_double2(f[y] * inv, 0.0);
  out[2 * NN + e] = make_double2(f[z] * inv, 0.0);
  out[3 * NN + e] = make_double2(f2[x] * inv, 0.0);
  out[4 * NN + e] = make_double2(f2[y] * inv, 0.0);
  out[5 * NN + e] = make_double2(f2[z] * inv, 0.0);
}

// The same on the 2^n x 2^n grid (plane problems): 4 x 2^(2n) entries,
// control (sigma, a), a in {x, y}
__global__ void k_direction2d(const double* __restrict__ f, const double* __restrict__ f2, int n, long NN,
                              cplx* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NN) return;
  const int N = 1 << n;
  const int x = (int)(e >> n), y = (int)(e & (N - 1));
  const double r2 = f[x] * f[x] + f[y] * f[y];
  const double inv = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
  out[0 * NN + e] = make_double2(f[x] * inv, 0.0);
  out[1 * NN + e] = make_double2(f[y] * inv, 0.0);
  out[2 * NN + e] = make_double2(f2[x] * inv, 0.0);
  out[3 * NN + e] = make_double2(f2[y] * inv, 0.0);
}

void direction2d(const double* f, const double* f2, int n, cplx* out, hipStream_t s) {
  const long NN = 1L << (2 * n);
  hipLaunchKernelGGL(k_direction2d, dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, s, f, f2, n, NN, out);
  check(hipGetLastError(), "direction2d launch");
}

void direction(const double* f, const double* f2, int n, cplx* out, hipStream_t s) {
  const long NN = 1L << (3 * n);
  hipLaunchKernelGGL(k_direction, dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, s, f, f2, n, NN, out);
  check(hipGetLastError(), "direction launch");
}

// Staggered-grid directions (App. A, Table 3): per axis the forward and
// backward difference symbols kp, km of the momentum index; out[a] =
// kp_a / |kp|, out[3 + a] = km_a / |kp| (|km| = |kp| per axis), 0 at the
// zero frequency
__global__ void k_direction_staggered(const cplx* __restrict__ kp, const cplx* __restrict__ km, int n, long NN,
                                      cplx* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NN) return;
  const int N = 1 << n;
  const int ix[3] = {(int)(e >> (2 * n)), (int)((e >> n) & (N - 1)), (int)(e & (N - 1))};
  double r2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) r2 += kp[ix[a]].x * kp[ix[a]].x + kp[ix[a]].y * kp[ix[a]].y;
  const double inv = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    out[a * NN + e] = make_double2(kp[ix[a]].x * inv, kp[ix[a]].y * inv);
    out[(3 + a) * NN + e] = make_double2(km[ix[a]].x * inv, km[ix[a]].y * inv);
  }
}

// The plane version: 4 x 2^(2n) entries, control (t, a), a in {x, y}
__global__ void k_direction_staggered2d(const cplx* __restrict__ kp, const cplx* __restrict__ km, int n, long NN,
                                        cplx* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NN) return;
  const int N = 1 << n;
  const int ix[2] = {(int)(e >> n), (int)(e & (N - 1))};
  double r2 = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a) r2 += kp[ix[a]].x * kp[ix[a]].x + kp[ix[a]].y * kp[ix[a]].y;
  const double inv = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    out[a * NN + e] = make_double2(kp[ix[a]].x * inv, kp[ix[a]].y * inv);
    out[(2 + a) * NN + e] = make_double2(km[ix[a]].x * inv, km[ix[a]].y * inv);
  }
}

void direction_staggered2d(const cplx* kp, const cplx* km, int n, cplx* out, hipStream_t s) {
  const long NN = 1L << (2 * n);
  hipLaunchKernelGGL(k_direction_staggered2d, dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, s, kp, km, n, NN,
                     out);
  check(hipGetLastError(), "direction_staggered2d launch");
}

void direction_staggered(const cplx* kp, const cplx* km, int n, cplx* out, hipStream_t s) {
  const long NN = 1L << (3 * n);
  hipLaunchKernelGGL(k_direction_staggered, dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, s, kp, km, n, NN,
                     out);
  check(hipGetLastError(), "direction_staggered launch");
}

// Majority phase of every 2 x 2 x 2 block of an N^3 phase array (C order,
// x slowest) -> (N/2)^3; ties go to the lowest phase id.  Ids >= nphase
// (at most 16) count as phase 0 here; the one-hot pass of the coarse array
// rejects nothing then, the fine array's own pass flags them.
__global__ void k_coarsen_majority(const uint8_t* __restrict__ phase, int n, int nphase,
                                   uint8_t* __restrict__ out) {
  const int h = n - 1, H = 1 << h, N = 1 << n;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (1L << (3 * h))) return;
  const int x = (int)(e >> (2 * h)), y = (int)((e >> h) & (H - 1)), z = (int)(e & (H - 1));
  int cnt[16];
#pragma unroll
  for (int p = 0; p < 16; ++p) cnt[p] = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const long f = ((long)(2 * x + (c >> 2)) * N + (2 * y + ((c >> 1) & 1))) * N + (2 * z + (c & 1));
    const int p = phase[f];
#pragma unroll
    for (int q = 0; q < 16; ++q) cnt[q] += (q == (p < nphase ? p : 0));
  }
  int best = 0;
#pragma unroll
  for (int q = 1; q < 16; ++q) best = cnt[q] > cnt[best] ? q : best;
  out[e] = (uint8_t)best;
}

// The same on an N x N pixel grid (plane geometries): 2 x 2 blocks.
__global__ void k_coarsen_majority2d(const uint8_t* __restrict__ phase, int n, int nphase,
                                     uint8_t* __restrict__ out) {
  const int h = n - 1, H = 1 << h, N = 1 << n;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (1L << (2 * h))) return;
  const int x = (int)(e >> h), y = (int)(e & (H - 1));
  int cnt[16];
#pragma unroll
  for (int p = 0; p < 16; ++p) cnt[p] = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const long f = (long)(2 * x + (c >> 1)) * N + (2 * y + (c & 1));
    const int p = phase[f];
#pragma unroll
    for (int q = 0; q < 16; ++q) cnt[q] += (q == (p < nphase ? p : 0));
  }
  int best = 0;
#pragma unroll
  for (int q = 1; q < 16; ++q) best = cnt[q] > cnt[best] ? q : best;
  out[e] = (uint8_t)best;
}

void coarsen_majority(const uint8_t* phase, int n, int nphase, uint8_t* out, hipStream_t s, int dim) {
  const long M = 1L << (dim * (n - 1));
  if (dim == 2)
    hipLaunchKernelGGL(k_coarsen_majority2d, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, phase, n, nphase,
                       out);
  else
    hipLaunchKernelGGL(k_coarsen_majority, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, phase, n, nphase,
                       out);
  check(hipGetLastError(), "coarsen launch");
}

__global__ void k_sum_middle(long total, int outer, int np, int inner, const cplx* in,
                             cplx* out, cplx w) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int c = e % inner;
  const long bo = e / inner;
  const cplx* p = in + bo * (long)np * inner + c;
  cplx acc = make_double2(0.0, 0.0);
  for (int q = 0; q < np; ++q) acc = cadd(acc, p[(long)q * inner]);
  out[e] = cmul(w, acc);
}

void sum_middle(int batch, int outer, int np, int inner, const cplx* in, cplx* out, cplx w,
                hipStream_t s) {
  const long total = (long)batch * outer * inner;
  if (total == 0) return;
  hipLaunchKernelGGL(k_sum_middle, dim3((total + 255) / 256), dim3(256), 0, s, total, outer,
                     np, inner, in, out, w);
  check(hipGetLastError(), "sum_middle launch");
}

}  // namespace qtt
