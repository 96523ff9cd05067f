// Complex FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64).
//
// One workgroup computes a 64 x 64 complex tile of C with 4 waves (2 x 2),
// each wave a 32 x 32 sub-tile made of 2 x 2 MFMA blocks of 16 x 16.  The
// complex product is four real MFMAs per block (re*re, -im*im, re*im,
// im*re) into separate real and imaginary accumulators.  A and B stage
// through LDS in split real/imaginary planes, 16 complex values of K per
// stage; the next stage is fetched into registers while the matrix cores
// work on the current one.  Operand lane layout of the 16x16x4 FP64
// instruction:
//   A: lane l holds A[l % 16][l / 16];  B: lane l holds B[l / 16][l % 16];
//   D: lane l, register r holds D[4 r + l / 16][l % 16].
//
// Shapes with few output tiles and a long contraction (the sketch products
// of TT-rounding: 160 x 80 outputs over K = 800) split K over workgroups;
// each slice writes its partial sums to a workspace and a second kernel
// adds the slices in fixed order (deterministic) and applies alpha, beta.
#include "qtt_internal.h"

#include <algorithm>
#include <stdexcept>

namespace qtt {

namespace {

typedef double dv4 __attribute__((ext_vector_type(4)));
typedef float fv4 __attribute__((ext_vector_type(4)));

constexpr int MT = 64, NT = 64, KT = 16;
constexpr int PAD = 2;
constexpr int NTHR = 256;
constexpr int PER_T = MT * KT / NTHR;  // staged elements per thread and operand (4)

// FP64 kernel over a WM x WN grid of waves, each wave BM x BN MFMA blocks
// of 16 x 16: 64 x 64 tiles (2 x 2 waves of 2 x 2 blocks) for large outputs,
// 32 x 32 tiles (2 x 2 waves of one block) when 64 x 64 tiles would leave
// compute units idle.
template <int WM, int WN, int BM, int BN>
__global__ __launch_bounds__(64 * WM * WN) void k_zgemm_mfma(GemmArgs g, int ksplit, int kchunk) {
  constexpr int MT = 16 * BM * WM, NT = 16 * BN * WN, NTHR = 64 * WM * WN;
  constexpr int PER_TA = MT * KT / NTHR, PER_TB = NT * KT / NTHR;
  __shared__ double Ar[KT][MT + PAD], Ai[KT][MT + PAD];
  __shared__ double Br[KT][NT + PAD], Bi[KT][NT + PAD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w / WN, wn = w % WN;   // wave position in the grid
  const int m0 = blockIdx.y * MT, n0 = blockIdx.x * NT;
  const int bz = blockIdx.z / ksplit, slice = blockIdx.z % ksplit;
  long oa, ob, oc;
  gemm_batch_offsets(g, bz, oa, ob, oc);
  const cplx* A = g.A + oa;
  const cplx* B = g.B + ob;
  const int kbeg = slice * kchunk, kend = min(g.K, kbeg + kchunk);

  dv4 cr[BM][BN], ci[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      cr[i][j] = dv4{0.0, 0.0, 0.0, 0.0};
      ci[i][j] = dv4{0.0, 0.0, 0.0, 0.0};
    }

  cplx ra[PER_TA], rb[PER_TB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int t = 0; t < PER_TA; ++t) {
      const int e = tid + NTHR * t;
      int mm, kk;
      if (g.opA == OP_N) { kk = e % KT; mm = e / KT; }
      else { mm = e % MT; kk = e / MT; }
      const int m = m0 + mm, k = k0 + kk;
      cplx v = make_double2(0.0, 0.0);
      if (m < g.M && k < kend) {
        if (g.opA == OP_N) v = A[(long)m * g.lda + k];
        else {
          v = A[(long)k * g.lda + m];
          if (g.opA == OP_C) v.y = -v.y;
        }
      }
      ra[t] = v;
    }
#pragma unroll
    for (int t = 0; t < PER_TB; ++t) {
      const int e = tid + NTHR * t;
      int nn, kk;
      if (g.opB == OP_N) { nn = e % NT; kk = e / NT; }
      else { kk = e % KT; nn = e / KT; }
      const int n = n0 + nn, k = k0 + kk;
      cplx v = make_double2(0.0, 0.0);
      if (n < g.N && k < kend) {
        if (g.opB == OP_N) v = B[(long)k * g.ldb + n];
        else {
          v = B[(long)n * g.ldb + k];
          if (g.opB == OP_C) v.y = -v.y;
        }
      }
      rb[t] = v;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int t = 0; t < PER_TA; ++t) {
      const int e = tid + NTHR * t;
      int mm, kk;
      if (g.opA == OP_N) { kk = e % KT; mm = e / KT; }
      else { mm = e % MT; kk = e / MT; }
      Ar[kk][mm] = ra[t].x;
      Ai[kk][mm] = ra[t].y;
    }
#pragma unroll
    for (int t = 0; t < PER_TB; ++t) {
      const int e = tid + NTHR * t;
      int nn, kk;
      if (g.opB == OP_N) { nn = e % NT; kk = e / NT; }
      else { kk = e % KT; nn = e / KT; }
      Br[kk][nn] = rb[t].x;
      Bi[kk][nn] = rb[t].y;
    }
  };

  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += KT) {
    stage();
    __syncthreads();
    if (k0 + KT < kend) fetch(k0 + KT);  // in flight during the MFMAs below
#pragma unroll
    for (int k4 = 0; k4 < KT / 4; ++k4) {
      const int kk = k4 * 4 + (lane >> 4);
      double ar[BM], ai[BM], nai[BM], br[BN], bi[BN];
#pragma unroll
      for (int i = 0; i < BM; ++i) {
        const int mm = wm * 16 * BM + i * 16 + (lane & 15);
        ar[i] = Ar[kk][mm];
        ai[i] = Ai[kk][mm];
        nai[i] = -ai[i];
      }
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        const int nn = wn * 16 * BN + j * 16 + (lane & 15);
        br[j] = Br[kk][nn];
        bi[j] = Bi[kk][nn];
      }
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], cr[i][j], 0, 0, 0);
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[i], bi[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], ci[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], ci[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }

  if (ksplit > 1) {
    // raw partial sums of this K slice: ws[slice][bz][m][n]
    cplx* P = g.ws + ((long)slice * gemm_nbatch(g) + bz) * (long)g.M * g.N;
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm * 16 * BM + i * 16 + 4 * r + (lane >> 4);
          const int n = n0 + wn * 16 * BN + j * 16 + (lane & 15);
          if (m < g.M && n < g.N) P[(long)m * g.N + n] = make_double2(cr[i][j][r], ci[i][j][r]);
        }
    return;
  }
  cplx* C = g.C + oc;
  const bool zb = (g.beta.x == 0.0 && g.beta.y == 0.0);
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 16 * BM + i * 16 + 4 * r + (lane >> 4);
        const int n = n0 + wn * 16 * BN + j * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        const double re = cr[i][j][r], im = ci[i][j][r];
        cplx out = make_double2(g.alpha.x * re - g.alpha.y * im, g.alpha.x * im + g.alpha.y * re);
        cplx* cp = C + (long)m * g.ldc + n;
        if (!zb) {
          const cplx c0 = *cp;
          out.x += g.beta.x * c0.x - g.beta.y * c0.y;
          out.y += g.beta.x * c0.y + g.beta.y * c0.x;
        }
        *cp = out;
      }
}

// The same tiling with FP32 operands and FP32 accumulation on
// v_mfma_f32_16x16x4f32 (twice the FP64 matrix rate): operands are rounded
// to float when staged, results widened to double on store.  Output lane
// layout of this instruction: lane l, register r holds D[4 (l / 16) + r][l % 16].
__global__ __launch_bounds__(NTHR) void k_zgemm_mfma32(GemmArgs g, int ksplit, int kchunk) {
  __shared__ float Ar[KT][MT + 4], Ai[KT][MT + 4];
  __shared__ float Br[KT][NT + 4], Bi[KT][NT + 4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int m0 = blockIdx.y * MT, n0 = blockIdx.x * NT;
  const int bz = blockIdx.z / ksplit, slice = blockIdx.z % ksplit;
  long oa, ob, oc;
  gemm_batch_offsets(g, bz, oa, ob, oc);
  const cplx* A = g.A + oa;
  const cplx* B = g.B + ob;
  const int kbeg = slice * kchunk, kend = min(g.K, kbeg + kchunk);

  fv4 cr[2][2], ci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cr[i][j] = fv4{0.f, 0.f, 0.f, 0.f};
      ci[i][j] = fv4{0.f, 0.f, 0.f, 0.f};
    }
  cplx ra[PER_T], rb[PER_T];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int t = 0; t < PER_T; ++t) {
      const int e = tid + NTHR * t;
      int mm, kk;
      if (g.opA == OP_N) { kk = e % KT; mm = e / KT; }
      else { mm = e % MT; kk = e / MT; }
      const int m = m0 + mm, k = k0 + kk;
      cplx v = make_double2(0.0, 0.0);
      if (m < g.M && k < kend) {
        if (g.opA == OP_N) v = A[(long)m * g.lda + k];
        else {
          v = A[(long)k * g.lda + m];
          if (g.opA == OP_C) v.y = -v.y;
        }
      }
      ra[t] = v;
    }
#pragma unroll
    for (int t = 0; t < PER_T; ++t) {
      const int e = tid + NTHR * t;
      int nn, kk;
      if (g.opB == OP_N) { nn = e % NT; kk = e / NT; }
      else { kk = e % KT; nn = e / KT; }
      const int n = n0 + nn, k = k0 + kk;
      cplx v = make_double2(0.0, 0.0);
      if (n < g.N && k < kend) {
        if (g.opB == OP_N) v = B[(long)k * g.ldb + n];
        else {
          v = B[(long)n * g.ldb + k];
          if (g.opB == OP_C) v.y = -v.y;
        }
      }
      rb[t] = v;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int t = 0; t < PER_T; ++t) {
      const int e = tid + NTHR * t;
      int mm, kk;
      if (g.opA == OP_N) { kk = e % KT; mm = e / KT; }
      else { mm = e % MT; kk = e / MT; }
      Ar[kk][mm] = (float)ra[t].x;
      Ai[kk][mm] = (float)ra[t].y;
    }
#pragma unroll
    for (int t = 0; t < PER_T; ++t) {
      const int e = tid + NTHR * t;
      int nn, kk;
      if (g.opB == OP_N) { nn = e % NT; kk = e / NT; }
      else { kk = e % KT; nn = e / KT; }
      Br[kk][nn] = (float)rb[t].x;
      Bi[kk][nn] = (float)rb[t].y;
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += KT) {
    stage();
    __syncthreads();
    if (k0 + KT < kend) fetch(k0 + KT);
#pragma unroll
    for (int k4 = 0; k4 < KT / 4; ++k4) {
      const int kk = k4 * 4 + (lane >> 4);
      float ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int mm = wm * 32 + i * 16 + (lane & 15);
        ar[i] = Ar[kk][mm];
        ai[i] = Ai[kk][mm];
        nai[i] = -ai[i];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int nn = wn * 32 + j * 16 + (lane & 15);
        br[j] = Br[kk][nn];
        bi[j] = Bi[kk][nn];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], br[j], cr[i][j], 0, 0, 0);
          cr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai[i], bi[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], bi[j], ci[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i], br[j], ci[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  if (ksplit > 1) {
    cplx* P = g.ws + ((long)slice * gemm_nbatch(g) + bz) * (long)g.M * g.N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
          const int n = n0 + wn * 32 + j * 16 + (lane & 15);
          if (m < g.M && n < g.N) P[(long)m * g.N + n] = make_double2(cr[i][j][r], ci[i][j][r]);
        }
    return;
  }
  cplx* C = g.C + oc;
  const bool zb = (g.beta.x == 0.0 && g.beta.y == 0.0);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        const double re = cr[i][j][r], im = ci[i][j][r];
        cplx out = make_double2(g.alpha.x * re - g.alpha.y * im, g.alpha.x * im + g.alpha.y * re);
        cplx* cp = C + (long)m * g.ldc + n;
        if (!zb) {
          const cplx c0 = *cp;
          out.x += g.beta.x * c0.x - g.beta.y * c0.y;
          out.y += g.beta.x * c0.y + g.beta.y * c0.x;
        }
        *cp = out;
      }
}

// C = alpha * sum_s ws[s] + beta * C, slices added in order s = 0, 1, ...
__global__ __launch_bounds__(256) void k_zgemm_reduce(GemmArgs g, int ksplit) {
  const long mn = (long)g.M * g.N, nb = gemm_nbatch(g);
  const long total = nb * mn;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256L) {
    const long bz = e / mn, r = e % mn;
    const int m = (int)(r / g.N), n = (int)(r % g.N);
    double sx = 0.0, sy = 0.0;
    for (int s = 0; s < ksplit; ++s) {
      const cplx p = g.ws[((long)s * nb + bz) * mn + r];
      sx += p.x;
      sy += p.y;
    }
    long oa, ob, oc;
    gemm_batch_offsets(g, bz, oa, ob, oc);
    cplx* cp = g.C + oc + (long)m * g.ldc + n;
    cplx out = make_double2(g.alpha.x * sx - g.alpha.y * sy, g.alpha.x * sy + g.alpha.y * sx);
    if (g.beta.x != 0.0 || g.beta.y != 0.0) {
      const cplx c0 = *cp;
      out.x += g.beta.x * c0.x - g.beta.y * c0.y;
      out.y += g.beta.x * c0.y + g.beta.y * c0.x;
    }
    *cp = out;
  }
}

}  // namespace

bool gemm_mfma_ok(int M, int N, int K) { return M >= 32 && N >= 32 && K >= 8 && (M + 31) / 32 <= 65535; }

// tile of the FP64 path: 32 x 32 (one wave) when 64 x 64 tiles would give
// fewer than two workgroups per compute unit
static bool small_tiles(int M, int N, long nbatch) {
  const long tiles64 = (long)((M + 63) / 64) * ((N + 63) / 64) * nbatch;
  return tiles64 < 512;
}

int gemm_ksplit(int M, int N, int K, long nbatch) {
  if (!gemm_mfma_ok(M, N, K)) return 1;
  const bool sm = small_tiles(M, N, nbatch);
  const int t = sm ? 32 : 64;
  const long tiles = (long)((M + t - 1) / t) * ((N + t - 1) / t) * nbatch;
  const long want = sm ? 1024 : 512;   // workgroups to aim at (4 waves each)
  if (tiles >= want / 2 || K < 4 * KT) return 1;
  // every slice at least 2 stages of K
  long s = std::min<long>((want + tiles - 1) / tiles, K / (2 * KT));
  s = std::min<long>(s, 32);
  if (tiles * s > 65535) s = 65535 / tiles;
  return (int)std::max<long>(1, s);
}

size_t gemm_ws_elems(const GemmArgs& g, int ksplit) {
  return ksplit > 1 ? (size_t)ksplit * gemm_nbatch(g) * (size_t)g.M * g.N : 0;
}

bool gemm_mfma(const GemmArgs& g, hipStream_t s) {
  if (!gemm_mfma_ok(g.M, g.N, g.K)) return false;
  int ks = g.ksplit > 1 && g.ws ? g.ksplit : 1;
  const long nb = gemm_nbatch(g);
  if (nb * ks > 65535) ks = 1;
  // slice length: a multiple of the stage depth
  const int per = (g.K + ks - 1) / ks;
  const int kchunk = (per + KT - 1) / KT * KT;
  ks = (g.K + kchunk - 1) / kchunk;
  if (g.fp32) {
    dim3 grid((g.N + NT - 1) / NT, (g.M + MT - 1) / MT, (unsigned)(nb * ks));
    if (grid.y > 65535u) return false;
    hipLaunchKernelGGL(k_zgemm_mfma32, grid, dim3(NTHR), 0, s, g, ks, kchunk);
  } else if (small_tiles(g.M, g.N, nb)) {
    dim3 grid((g.N + 31) / 32, (g.M + 31) / 32, (unsigned)(nb * ks));
    hipLaunchKernelGGL((k_zgemm_mfma<2, 2, 1, 1>), grid, dim3(256), 0, s, g, ks, kchunk);
  } else {
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, (unsigned)(nb * ks));
    hipLaunchKernelGGL((k_zgemm_mfma<2, 2, 2, 2>), grid, dim3(256), 0, s, g, ks, kchunk);
  }
  check(hipGetLastError(), "zgemm_mfma launch");
  if (ks > 1) {
    const long total = nb * g.M * (long)g.N;
    const long blocks = std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zgemm_reduce, dim3((unsigned)blocks), dim3(256), 0, s, g, ks);
    check(hipGetLastError(), "zgemm_reduce launch");
  }
  return true;
}

}  // namespace qtt
