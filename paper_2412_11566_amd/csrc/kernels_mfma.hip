// Complex FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64).
//
// One workgroup computes a 64 x 64 complex tile of C with 4 waves (2 x 2),
// each wave a 32 x 32 sub-tile made of 2 x 2 MFMA blocks of 16 x 16.  The
// complex product is four real MFMAs per block (re*re, -im*im, re*im,
// im*re) into separate real and imaginary accumulators.  A and B stage
// through LDS in split real/imaginary planes, 16 complex values of K per
// stage.  Operand lane layout of the 16x16x4 FP64 instruction:
//   A: lane l holds A[l % 16][l / 16];  B: lane l holds B[l / 16][l % 16];
//   D: lane l, register r holds D[4 r + l / 16][l % 16].
#include "qtt_internal.h"

#include <stdexcept>

namespace qtt {

namespace {

typedef double dv4 __attribute__((ext_vector_type(4)));

constexpr int MT = 64, NT = 64, KT = 16;
constexpr int PAD = 2;

__global__ __launch_bounds__(256) void k_zgemm_mfma(GemmArgs g) {
  __shared__ double Ar[KT][MT + PAD], Ai[KT][MT + PAD];
  __shared__ double Br[KT][NT + PAD], Bi[KT][NT + PAD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;   // wave position in the 2 x 2 grid
  const int m0 = blockIdx.y * MT, n0 = blockIdx.x * NT;
  const int bz = blockIdx.z;
  const int b1 = bz / g.nb2, b2 = bz % g.nb2;
  const cplx* A = g.A + b1 * g.sA1 + b2 * g.sA2;
  const cplx* B = g.B + b1 * g.sB1 + b2 * g.sB2;
  cplx* C = g.C + b1 * g.sC1 + b2 * g.sC2;

  dv4 cr[2][2], ci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cr[i][j] = dv4{0.0, 0.0, 0.0, 0.0};
      ci[i][j] = dv4{0.0, 0.0, 0.0, 0.0};
    }

  for (int k0 = 0; k0 < g.K; k0 += KT) {
    // stage A (MT x KT) and B (KT x NT)
    for (int e = tid; e < MT * KT; e += 256) {
      int mm, kk;
      if (g.opA == OP_N) { kk = e % KT; mm = e / KT; }
      else { mm = e % MT; kk = e / MT; }
      const int m = m0 + mm, k = k0 + kk;
      cplx v = make_double2(0.0, 0.0);
      if (m < g.M && k < g.K) {
        if (g.opA == OP_N) v = A[(long)m * g.lda + k];
        else {
          v = A[(long)k * g.lda + m];
          if (g.opA == OP_C) v.y = -v.y;
        }
      }
      Ar[kk][mm] = v.x;
      Ai[kk][mm] = v.y;
    }
    for (int e = tid; e < NT * KT; e += 256) {
      int nn, kk;
      if (g.opB == OP_N) { nn = e % NT; kk = e / NT; }
      else { kk = e % KT; nn = e / KT; }
      const int n = n0 + nn, k = k0 + kk;
      cplx v = make_double2(0.0, 0.0);
      if (n < g.N && k < g.K) {
        if (g.opB == OP_N) v = B[(long)k * g.ldb + n];
        else {
          v = B[(long)n * g.ldb + k];
          if (g.opB == OP_C) v.y = -v.y;
        }
      }
      Br[kk][nn] = v.x;
      Bi[kk][nn] = v.y;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < KT / 4; ++k4) {
      const int kk = k4 * 4 + (lane >> 4);
      double ar[2], ai[2], nai[2], br[2], bi[2];
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
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], cr[i][j], 0, 0, 0);
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[i], bi[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], ci[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], ci[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  const bool zb = (g.beta.x == 0.0 && g.beta.y == 0.0);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 32 + i * 16 + 4 * r + (lane >> 4);
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

}  // namespace

bool gemm_mfma(const GemmArgs& g, hipStream_t s) {
  if (g.M < 32 || g.N < 32 || g.K < 8) return false;
  dim3 grid((g.N + NT - 1) / NT, (g.M + MT - 1) / MT, g.nb1 * g.nb2);
  if (grid.x > 2147483647u || grid.y > 65535u) return false;
  hipLaunchKernelGGL(k_zgemm_mfma, grid, dim3(256), 0, s, g);
  check(hipGetLastError(), "zgemm_mfma launch");
  return true;
}

}  // namespace qtt
