// Complex FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64).
//
// One workgroup computes a complex tile of C with a grid of waves, each
// wave a sub-tile of 16 x 16 MFMA blocks (tiles from 16 x 16 to 80 x 80,
// chosen per shape to limit padding and fill the compute units).  The
// complex product is three real MFMAs per block where the registers hold a
// third accumulator (Gauss: re*re, im*im and (re+im)*(re+im), combined
// after the contraction), four otherwise.  A and B stage
// through LDS in split real/imaginary planes, 16 complex values of K per
// stage; the next stage is fetched into registers while the matrix cores
// work on the current one.  Operand lane layout of the 16x16x4 FP64
// instruction:
//   A: lane l holds A[l % 16][l / 16];  B: lane l holds B[l / 16][l % 16];
//   D: lane l, register r holds D[4 r + l / 16][l % 16].
//
// Shapes with few output tiles and a long contraction (the sketch products
// of TT-rounding: 160 x 80 outputs over K = 12240) split K over workgroups;
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

// span of a timed launch (GemmArgs::span, null otherwise): the earliest
// workgroup start and the latest workgroup end on the device's
// constant-rate real-time counter; the end is taken after the whole
// workgroup has issued its stores
__device__ __forceinline__ void span_begin(unsigned long long* t) {
  if (t && threadIdx.x == 0) atomicMin(t, (unsigned long long)wall_clock64());
}
__device__ __forceinline__ void span_end(unsigned long long* t) {
  if (t) {
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(t + 1, (unsigned long long)wall_clock64());
  }
}

// FP64 kernel over a WM x WN grid of waves, each wave BM x BN MFMA blocks
// of 16 x 16 (tile variants and their choice: plan_fp64 below).
template <int WM, int WN, int BM, int BN, bool G3>
__global__ __launch_bounds__(64 * WM * WN, 2) void k_zgemm_mfma(GemmArgs g, int ksplit, int kchunk) {
  constexpr int MT = 16 * BM * WM, NT = 16 * BN * WN, NTHR = 64 * WM * WN;
  constexpr int PER_TA = MT * KT / NTHR, PER_TB = NT * KT / NTHR;
  __shared__ double Ar[KT][MT + PAD], Ai[KT][MT + PAD];
  __shared__ double Br[KT][NT + PAD], Bi[KT][NT + PAD];
  span_begin(g.span);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w / WN, wn = w % WN;   // wave position in the grid
  const int m0 = blockIdx.y * MT, n0 = blockIdx.x * NT;
  const int bz = blockIdx.z / ksplit, slice = blockIdx.z % ksplit;
  long oa, ob, oc;
  gemm_batch_offsets(g, bz, oa, ob, oc);
  const cplx* A = g.A + oa;
  const cplx* B = g.B + ob;
  const int kbeg = slice * kchunk, kend = min(g.K, kbeg + kchunk);

  // G3: three real products per complex block (Gauss): cr = Ar Br,
  // c2 = Ai Bi, ci = (Ar + Ai)(Br + Bi); then Re C = cr - c2,
  // Im C = ci - cr - c2.  Otherwise four: cr = Ar Br - Ai Bi,
  // ci = Ar Bi + Ai Br (one accumulator fewer per block, for the variants
  // whose registers cannot hold a third)
  dv4 cr[BM][BN], ci[BM][BN], c2[G3 ? BM : 1][G3 ? BN : 1];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      cr[i][j] = dv4{0.0, 0.0, 0.0, 0.0};
      ci[i][j] = dv4{0.0, 0.0, 0.0, 0.0};
      if (G3) c2[G3 ? i : 0][G3 ? j : 0] = dv4{0.0, 0.0, 0.0, 0.0};
    }

  // fetch: raw loads only (indices clamped in range, validity kept in a
  // mask) so no load waits on its data before the stage that stores it;
  // stage: mask, conjugate and split into the LDS planes
  cplx ra[PER_TA], rb[PER_TB];
  unsigned oka = 0u, okb = 0u;
  auto fetch = [&](int k0) {
    oka = 0u;
    okb = 0u;
#pragma unroll
    for (int t = 0; t < PER_TA; ++t) {
      const int e = tid + NTHR * t;
      int mm, kk;
      if (g.opA == OP_N) { kk = e % KT; mm = e / KT; }
      else { mm = e % MT; kk = e / MT; }
      const int m = m0 + mm, k = k0 + kk;
      const bool ok = m < g.M && k < kend;
      const long idx = g.opA == OP_N ? (long)m * g.lda + k : (long)k * g.lda + m;
      ra[t] = A[ok ? idx : 0];
      oka |= ok ? (1u << t) : 0u;
    }
#pragma unroll
    for (int t = 0; t < PER_TB; ++t) {
      const int e = tid + NTHR * t;
      int nn, kk;
      if (g.opB == OP_N) { nn = e % NT; kk = e / NT; }
      else { kk = e % KT; nn = e / KT; }
      const int n = n0 + nn, k = k0 + kk;
      const bool ok = n < g.N && k < kend;
      const long idx = g.opB == OP_N ? (long)k * g.ldb + n : (long)n * g.ldb + k;
      rb[t] = B[ok ? idx : 0];
      okb |= ok ? (1u << t) : 0u;
    }
  };
  const double sa = g.opA == OP_C ? -1.0 : 1.0, sb = g.opB == OP_C ? -1.0 : 1.0;
  auto stage = [&]() {
#pragma unroll
    for (int t = 0; t < PER_TA; ++t) {
      const int e = tid + NTHR * t;
      int mm, kk;
      if (g.opA == OP_N) { kk = e % KT; mm = e / KT; }
      else { mm = e % MT; kk = e / MT; }
      const bool ok = (oka >> t) & 1u;
      Ar[kk][mm] = ok ? ra[t].x : 0.0;
      Ai[kk][mm] = ok ? sa * ra[t].y : 0.0;
    }
#pragma unroll
    for (int t = 0; t < PER_TB; ++t) {
      const int e = tid + NTHR * t;
      int nn, kk;
      if (g.opB == OP_N) { nn = e % NT; kk = e / NT; }
      else { kk = e % KT; nn = e / KT; }
      const bool ok = (okb >> t) & 1u;
      Br[kk][nn] = ok ? rb[t].x : 0.0;
      Bi[kk][nn] = ok ? sb * rb[t].y : 0.0;
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
      double ar[BM], ai[BM], sa[BM], br[BN], bi[BN], sb[BN];
#pragma unroll
      for (int i = 0; i < BM; ++i) {
        const int mm = wm * 16 * BM + i * 16 + (lane & 15);
        ar[i] = Ar[kk][mm];
        ai[i] = Ai[kk][mm];
        sa[i] = G3 ? ar[i] + ai[i] : -ai[i];
      }
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        const int nn = wn * 16 * BN + j * 16 + (lane & 15);
        br[j] = Br[kk][nn];
        bi[j] = Bi[kk][nn];
        sb[j] = G3 ? br[j] + bi[j] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], cr[i][j], 0, 0, 0);
          if (G3) {
            c2[G3 ? i : 0][G3 ? j : 0] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                ai[i], bi[j], c2[G3 ? i : 0][G3 ? j : 0], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[i], sb[j], ci[i][j], 0, 0, 0);
          } else {  // sa = -Ai
            cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[i], bi[j], cr[i][j], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], ci[i][j], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], ci[i][j], 0, 0, 0);
          }
        }
    }
    __syncthreads();
  }
  if (G3) {
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        const dv4 p2 = c2[G3 ? i : 0][G3 ? j : 0];
        ci[i][j] = ci[i][j] - cr[i][j] - p2;
        cr[i][j] = cr[i][j] - p2;
      }
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
    span_end(g.span);
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
  span_end(g.span);
}

// The same tiling with FP32 operands and FP32 accumulation on
// v_mfma_f32_16x16x4f32 (twice the FP64 matrix rate): operands are rounded
// to float when staged, results widened to double on store.  Output lane
// layout of this instruction: lane l, register r holds D[4 (l / 16) + r][l % 16].
__global__ __launch_bounds__(NTHR) void k_zgemm_mfma32(GemmArgs g, int ksplit, int kchunk) {
  __shared__ float Ar[KT][MT + 4], Ai[KT][MT + 4];
  __shared__ float Br[KT][NT + 4], Bi[KT][NT + 4];
  span_begin(g.span);
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
  // raw loads at fetch, mask / conjugate / round at stage (as in the FP64
  // kernel)
  cplx ra[PER_T], rb[PER_T];
  unsigned oka = 0u, okb = 0u;
  auto fetch = [&](int k0) {
    oka = 0u;
    okb = 0u;
#pragma unroll
    for (int t = 0; t < PER_T; ++t) {
      const int e = tid + NTHR * t;
      int mm, kk;
      if (g.opA == OP_N) { kk = e % KT; mm = e / KT; }
      else { mm = e % MT; kk = e / MT; }
      const int m = m0 + mm, k = k0 + kk;
      const bool ok = m < g.M && k < kend;
      const long idx = g.opA == OP_N ? (long)m * g.lda + k : (long)k * g.lda + m;
      ra[t] = A[ok ? idx : 0];
      oka |= ok ? (1u << t) : 0u;
    }
#pragma unroll
    for (int t = 0; t < PER_T; ++t) {
      const int e = tid + NTHR * t;
      int nn, kk;
      if (g.opB == OP_N) { nn = e % NT; kk = e / NT; }
      else { kk = e % KT; nn = e / KT; }
      const int n = n0 + nn, k = k0 + kk;
      const bool ok = n < g.N && k < kend;
      const long idx = g.opB == OP_N ? (long)k * g.ldb + n : (long)n * g.ldb + k;
      rb[t] = B[ok ? idx : 0];
      okb |= ok ? (1u << t) : 0u;
    }
  };
  const float sa = g.opA == OP_C ? -1.f : 1.f, sb = g.opB == OP_C ? -1.f : 1.f;
  auto stage = [&]() {
#pragma unroll
    for (int t = 0; t < PER_T; ++t) {
      const int e = tid + NTHR * t;
      int mm, kk;
      if (g.opA == OP_N) { kk = e % KT; mm = e / KT; }
      else { mm = e % MT; kk = e / MT; }
      const bool ok = (oka >> t) & 1u;
      Ar[kk][mm] = ok ? (float)ra[t].x : 0.f;
      Ai[kk][mm] = ok ? sa * (float)ra[t].y : 0.f;
    }
#pragma unroll
    for (int t = 0; t < PER_T; ++t) {
      const int e = tid + NTHR * t;
      int nn, kk;
      if (g.opB == OP_N) { nn = e % NT; kk = e / NT; }
      else { kk = e % KT; nn = e / KT; }
      const bool ok = (okb >> t) & 1u;
      Br[kk][nn] = ok ? (float)rb[t].x : 0.f;
      Bi[kk][nn] = ok ? sb * (float)rb[t].y : 0.f;
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
    span_end(g.span);
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
  span_end(g.span);
}

// Split-BF16 operands on v_mfma_f32_16x16x32_bf16 with FP32 accumulation
// (the contraction precision of QTT_PREC_BF16X3): every operand x is
// rounded to float and split as x = hi + lo, hi = bf16(x), lo =
// bf16(x - hi), so hi + lo carries 16 significant bits; each real product
// a b is formed as hi_a hi_b + hi_a lo_b + lo_a hi_b (the lo lo term, of
// relative size 2^-16, is dropped), three bf16 products per real product
// and twelve per complex block.  Same 64 x 64 tile and wave grid as the
// FP32 kernel, with K staged 32 at a time (one instruction's depth).
// Operands sit in LDS k-contiguous, one row of 32 (+ 8 pad) bf16 per tile
// row, so a lane's eight K values are one 16-byte read and the sixteen rows
// a quarter-wave reads fall in distinct banks (80-byte stride).  Lane
// layout of the instruction:
//   A: lane l holds A[l % 16][8 (l / 16) .. 8 (l / 16) + 7];
//   B: lane l holds B[8 (l / 16) .. 8 (l / 16) + 7][l % 16];
//   D: lane l, register r holds D[4 (l / 16) + r][l % 16].
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
constexpr int KB = 32, KBP = KB + 8;
constexpr int PER_B = MT * KB / NTHR;  // staged complex elements per thread and operand (8)

__device__ __forceinline__ void split_bf16(double x, __bf16& hi, __bf16& lo) {
  const float f = (float)x;
  hi = (__bf16)f;
  lo = (__bf16)(f - (float)hi);
}
__device__ __forceinline__ bf8 neg8(bf8 v) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  u4 b = __builtin_bit_cast(u4, v);
  b ^= 0x80008000u;
  return __builtin_bit_cast(bf8, b);
}

__global__ __launch_bounds__(NTHR) void k_zgemm_bf16x3(GemmArgs g, int ksplit, int kchunk) {
  // planes: 0 re hi, 1 re lo, 2 im hi, 3 im lo
  __shared__ __attribute__((aligned(16))) __bf16 As[4][MT][KBP];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[4][NT][KBP];
  span_begin(g.span);
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
  cplx ra[PER_B], rb[PER_B];
  unsigned oka = 0u, okb = 0u;
  // element e of a stage: A row mm / K index kk, B column nn / K index kk;
  // the K index runs fastest where the operand is K-contiguous in memory
  auto fetch = [&](int k0) {
    oka = 0u;
    okb = 0u;
#pragma unroll
    for (int t = 0; t < PER_B; ++t) {
      const int e = tid + NTHR * t;
      int mm, kk;
      if (g.opA == OP_N) { kk = e % KB; mm = e / KB; }
      else { mm = e % MT; kk = e / MT; }
      const int m = m0 + mm, k = k0 + kk;
      const bool ok = m < g.M && k < kend;
      const long idx = g.opA == OP_N ? (long)m * g.lda + k : (long)k * g.lda + m;
      ra[t] = A[ok ? idx : 0];
      oka |= ok ? (1u << t) : 0u;
    }
#pragma unroll
    for (int t = 0; t < PER_B; ++t) {
      const int e = tid + NTHR * t;
      int nn, kk;
      if (g.opB == OP_N) { nn = e % NT; kk = e / NT; }
      else { kk = e % KB; nn = e / KB; }
      const int n = n0 + nn, k = k0 + kk;
      const bool ok = n < g.N && k < kend;
      const long idx = g.opB == OP_N ? (long)k * g.ldb + n : (long)n * g.ldb + k;
      rb[t] = B[ok ? idx : 0];
      okb |= ok ? (1u << t) : 0u;
    }
  };
  const double sa = g.opA == OP_C ? -1.0 : 1.0, sb = g.opB == OP_C ? -1.0 : 1.0;
  auto stage = [&]() {
#pragma unroll
    for (int t = 0; t < PER_B; ++t) {
      const int e = tid + NTHR * t;
      int mm, kk;
      if (g.opA == OP_N) { kk = e % KB; mm = e / KB; }
      else { mm = e % MT; kk = e / MT; }
      const bool ok = (oka >> t) & 1u;
      __bf16 h, l;
      split_bf16(ok ? ra[t].x : 0.0, h, l);
      As[0][mm][kk] = h;
      As[1][mm][kk] = l;
      split_bf16(ok ? sa * ra[t].y : 0.0, h, l);
      As[2][mm][kk] = h;
      As[3][mm][kk] = l;
    }
#pragma unroll
    for (int t = 0; t < PER_B; ++t) {
      const int e = tid + NTHR * t;
      int nn, kk;
      if (g.opB == OP_N) { nn = e % NT; kk = e / NT; }
      else { kk = e % KB; nn = e / KB; }
      const bool ok = (okb >> t) & 1u;
      __bf16 h, l;
      split_bf16(ok ? rb[t].x : 0.0, h, l);
      Bs[0][nn][kk] = h;
      Bs[1][nn][kk] = l;
      split_bf16(ok ? sb * rb[t].y : 0.0, h, l);
      Bs[2][nn][kk] = h;
      Bs[3][nn][kk] = l;
    }
  };
  const int kq = 8 * (lane >> 4);
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += KB) {
    stage();
    __syncthreads();
    if (k0 + KB < kend) fetch(k0 + KB);
    bf8 a[2][4], b[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int mm = wm * 32 + i * 16 + (lane & 15);
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) a[i][pl] = *(const bf8*)&As[pl][mm][kq];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int nn = wn * 32 + j * 16 + (lane & 15);
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) b[j][pl] = *(const bf8*)&Bs[pl][nn][kq];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const bf8 nih = neg8(a[i][2]), nil = neg8(a[i][3]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        // re += Ar Br - Ai Bi;  im += Ar Bi + Ai Br  (hi hi, hi lo, lo hi each)
        fv4 r = cr[i][j], m = ci[i][j];
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][0], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][1], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], b[j][0], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, b[j][2], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, b[j][3], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nil, b[j][2], r, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][2], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][3], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], b[j][2], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], b[j][0], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], b[j][1], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][3], b[j][0], m, 0, 0, 0);
        cr[i][j] = r;
        ci[i][j] = m;
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
    span_end(g.span);
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
  span_end(g.span);
}

// C = alpha * sum_s ws[s] + beta * C, slices added in order s = 0, 1, ...
__global__ __launch_bounds__(256) void k_zgemm_reduce(GemmArgs g, int ksplit) {
  const long mn = (long)g.M * g.N, nb = gemm_nbatch(g);
  const long total = nb * mn;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256L) {
    const long bz = e / mn, r = e % mn;
    const int m = (int)(r / g.N), n = (int)(r % g.N);
    // partials summed in split order; four loads in flight per round
    double sx = 0.0, sy = 0.0;
    const cplx* wp = g.ws + bz * mn + r;
    const long step = nb * mn;
    int s = 0;
    for (; s + 4 <= ksplit; s += 4) {
      const cplx p0 = wp[(long)s * step], p1 = wp[(long)(s + 1) * step];
      const cplx p2 = wp[(long)(s + 2) * step], p3 = wp[(long)(s + 3) * step];
      sx += p0.x;
      sy += p0.y;
      sx += p1.x;
      sy += p1.y;
      sx += p2.x;
      sy += p2.y;
      sx += p3.x;
      sy += p3.y;
    }
    for (; s < ksplit; ++s) {
      const cplx p = wp[(long)s * step];
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

// FP64 tile variants (WM x WN waves of BM x BN blocks).  Sketch ranks of
// TT-rounding put 80 (cap 64 + oversampling 16) on one side of most
// products, which 80-wide tiles cover without padding; a wave then holds a
// 16 x 80 (or 80 x 16) strip of five blocks.
struct TileV {
  int wm, wn, bm, bn;
  bool g3;     // three real products per complex block (registers permitting)
  double eff;  // measured rate on padded work, relative units
  int mt() const { return 16 * bm * wm; }
  int nt() const { return 16 * bn * wn; }
  int waves() const { return wm * wn; }
};
constexpr TileV kTiles[] = {
    {1, 1, 1, 1, true, 3.0},     // 16 x 16
    {2, 2, 1, 1, true, 6.4},     // 32 x 32
    {2, 2, 2, 2, true, 7.0},     // 64 x 64
    {5, 1, 1, 5, true, 4.6},     // 80 x 80
    {2, 1, 1, 5, false, 5.3},    // 32 x 80
    {1, 2, 5, 1, false, 5.25},   // 80 x 32
    {4, 1, 1, 5, true, 7.7},     // 64 x 80
};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);
constexpr TileV kTileFp32 = {2, 2, 2, 2, false, 1.0};  // the FP32 kernel's fixed tile

bool gemm_mfma_ok(int M, int N, int K) { return M >= 16 && N >= 16 && K >= 4 && (M + 15) / 16 <= 65535; }

// workgroups whose waves fill the chip twice over (1024 SIMDs) need no K split
constexpr long kWaveTarget = 2048;

static int ksplit_for(const TileV& t, int M, int N, int K, long nbatch) {
  const long tiles = (long)((M + t.mt() - 1) / t.mt()) * ((N + t.nt() - 1) / t.nt()) * nbatch;
  const long waves = tiles * t.waves();
  if (waves >= kWaveTarget / 2 || K < 4 * KT) return 1;
  // every slice at least 2 stages of K
  long s = std::min<long>((kWaveTarget + waves - 1) / waves, K / (2 * KT));
  s = std::min<long>(s, 32);
  if (nbatch * s > 65535) s = 65535 / nbatch;
  return (int)std::max<long>(1, s);
}

struct Plan {
  int v;   // index into kTiles
  int ks;  // K slices
};

// The FP64 variant with the least modelled time: padded MFMA work over the
// waves that run it (up to two per SIMD) and over the variant's rate on
// padded work, measured on the batched products of TT-rounding (rank-80
// sketches against operator ranks of 60 to 160): 64 x 80 tiles with three
// products per block lead, 5-wave 80 x 80 tiles trail (one workgroup per
// compute unit at two waves per SIMD leaves one SIMD with two of its five
// waves).  Split-K shapes pay their padding twice: the padded slices also
// write and reduce partial sums.
static Plan plan_fp64(int M, int N, int K, long nbatch) {
  Plan best{2, 1};
  double bestc = 0.0;
  const double kp = (double)((K + KT - 1) / KT * KT);
  for (int v = 0; v < kNumTiles; ++v) {
    const TileV& t = kTiles[v];
    const long tm = (M + t.mt() - 1) / t.mt(), tn = (N + t.nt() - 1) / t.nt();
    if (tm > 65535 || tn > 65535) continue;
    const int ks = ksplit_for(t, M, N, K, nbatch);
    if (nbatch * ks > 65535) continue;
    const double work = (double)tm * t.mt() * (double)tn * t.nt() * kp * nbatch;
    const double waves = (double)tm * tn * nbatch * ks * t.waves();
    const double par = std::min(waves, (double)kWaveTarget);
    const double pad = (double)tm * t.mt() * tn * t.nt() / ((double)M * N);
    const double c = work / (par * t.eff) * (ks > 1 ? pad * pad : 1.0);
    if (bestc == 0.0 || c < bestc) {
      bestc = c;
      best = Plan{v, ks};
    }
  }
  return best;
}

int gemm_ksplit(int M, int N, int K, long nbatch, bool fp32, int tile) {
  if (!gemm_mfma_ok(M, N, K)) return 1;
  if (fp32) return ksplit_for(kTileFp32, M, N, K, nbatch);
  if (tile >= 0 && tile < kNumTiles) return ksplit_for(kTiles[tile], M, N, K, nbatch);
  return plan_fp64(M, N, K, nbatch).ks;
}
int gemm_num_tiles() { return kNumTiles; }

size_t gemm_ws_elems(const GemmArgs& g, int ksplit) {
  return ksplit > 1 ? (size_t)ksplit * gemm_nbatch(g) * (size_t)g.M * g.N : 0;
}

template <int WM, int WN, int BM, int BN, bool G3>
static void launch_fp64(const GemmArgs& g, int ks, int kchunk, hipStream_t s) {
  constexpr int MT = 16 * BM * WM, NT = 16 * BN * WN;
  dim3 grid((g.N + NT - 1) / NT, (g.M + MT - 1) / MT, (unsigned)(gemm_nbatch(g) * ks));
  hipLaunchKernelGGL((k_zgemm_mfma<WM, WN, BM, BN, G3>), grid, dim3(64 * WM * WN), 0, s, g, ks, kchunk);
}

bool gemm_mfma(const GemmArgs& g, hipStream_t s) {
  int ks = 1;
  if (!gemm_mfma_main(g, s, ks)) return false;
  gemm_mfma_reduce(g, ks, s);
  return true;
}

void gemm_mfma_reduce(const GemmArgs& g, int ks, hipStream_t s) {
  if (ks <= 1) return;
  const long total = gemm_nbatch(g) * g.M * (long)g.N;
  const long blocks = std::min<long>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zgemm_reduce, dim3((unsigned)blocks), dim3(256), 0, s, g, ks);
  check(hipGetLastError(), "zgemm_reduce launch");
}

bool gemm_mfma_main(const GemmArgs& g, hipStream_t s, int& ks_used) {
  ks_used = 1;
  if (!gemm_mfma_ok(g.M, g.N, g.K)) return false;
  const long nb = gemm_nbatch(g);
  const bool low = g.fp32 || g.bf16x3;
  Plan pl = low ? Plan{-1, 1} : plan_fp64(g.M, g.N, g.K, nb);
  if (!low && g.tile >= 0) {
    if (g.tile >= kNumTiles) return false;
    const TileV& t = kTiles[g.tile];
    if ((g.M + t.mt() - 1) / t.mt() > 65535 || (g.N + t.nt() - 1) / t.nt() > 65535) return false;
    pl.v = g.tile;
  }
  if ((g.fp32 || g.bf16x3) && (g.M + MT - 1) / MT > 65535) return false;
  // the split the caller sized the workspace for (gemm_ksplit), else none
  int ks = g.ksplit > 1 && g.ws ? g.ksplit : 1;
  if (nb * ks > 65535) ks = 1;
  // slice length: a multiple of the stage depth
  const int per = (g.K + ks - 1) / ks;
  const int kst = g.bf16x3 ? KB : KT;
  const int kchunk = (per + kst - 1) / kst * kst;
  ks = (g.K + kchunk - 1) / kchunk;
  if (g.bf16x3) {
    dim3 grid((g.N + NT - 1) / NT, (g.M + MT - 1) / MT, (unsigned)(nb * ks));
    hipLaunchKernelGGL(k_zgemm_bf16x3, grid, dim3(NTHR), 0, s, g, ks, kchunk);
  } else if (g.fp32) {
    dim3 grid((g.N + NT - 1) / NT, (g.M + MT - 1) / MT, (unsigned)(nb * ks));
    hipLaunchKernelGGL(k_zgemm_mfma32, grid, dim3(NTHR), 0, s, g, ks, kchunk);
  } else {
    switch (pl.v) {
      case 0: launch_fp64<1, 1, 1, 1, true>(g, ks, kchunk, s); break;
      case 1: launch_fp64<2, 2, 1, 1, true>(g, ks, kchunk, s); break;
      case 2: launch_fp64<2, 2, 2, 2, true>(g, ks, kchunk, s); break;
      case 3: launch_fp64<5, 1, 1, 5, true>(g, ks, kchunk, s); break;
      case 4: launch_fp64<2, 1, 1, 5, false>(g, ks, kchunk, s); break;
      case 5: launch_fp64<1, 2, 5, 1, false>(g, ks, kchunk, s); break;
      default: launch_fp64<4, 1, 1, 5, true>(g, ks, kchunk, s); break;
    }
  }
  check(hipGetLastError(), "zgemm_mfma launch");
  ks_used = ks;
  return true;
}

}  // namespace qtt
