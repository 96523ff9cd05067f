// Device tensor-train engine and C ABI of the qtthom library.
//
// Tensor trains live in HBM as rank-major cores (r_{k-1}, d_k, r_k); a
// handle may hold a batch of trains with common ranks (the six unit load
// cases of one structure).  Every product of an operator (TTO) with a
// train is followed by TT-rounding (Sec. 3 of the paper).  The rounding of
// a product is done without materialising it: a randomized range sketch of
// the implicit product (Gaussian tensor-train test vectors, contracted core
// by core right to left), a left-to-right QR sweep on the sketched
// unfoldings that yields a left-orthogonal train of the sketch ranks, and a
// right-to-left truncated-SVD sweep with the accuracy rule of
// eq. rounding_condition_tt.  When the sketch rank reaches the exact
// structural rank of every bond (QTT_EXACT, or no cap) the result is the
// exact product up to floating-point rounding before truncation.
#include "qtt_internal.h"
#include "host_ops.h"
#include "qtthom.h"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <thread>
#include <array>
#include <atomic>
#include <exception>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

namespace qtt {

// ---------------------------------------------------------------------------
// device memory pool (reuse on the context's single stream)
// ---------------------------------------------------------------------------
struct Pool {
  std::multimap<size_t, void*> freel;
  std::vector<void*> all;
  int device = 0;
  ~Pool() {
    for (void* p : all) (void)hipFree(p);
  }
  static size_t cls(size_t bytes) {
    size_t c = 256;
    while (c < bytes) c <<= 1;
    return c;
  }
  void* get(size_t bytes, size_t& c) {
    c = cls(bytes);
    auto it = freel.find(c);
    if (it != freel.end()) {
      void* p = it->second;
      freel.erase(it);
      return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, c) != hipSuccess) {
      // release cached blocks and retry once
      for (auto& kv : freel) {
        (void)hipFree(kv.second);
        all.erase(std::find(all.begin(), all.end(), kv.second));
      }
      freel.clear();
      if (hipMalloc(&p, c) != hipSuccess) throw std::bad_alloc();
    }
    all.push_back(p);
    return p;
  }
  void put(void* p, size_t c) { freel.emplace(c, p); }
  // live allocations (start -> requested bytes), for host-side bounds checks
  std::map<uintptr_t, size_t> live;
  // caller-owned device ranges wrapped as tensors (qtt_tensor_wrap); the
  // same range may be wrapped more than once
  std::multimap<uintptr_t, size_t> ext;
  bool contains(const void* p, size_t bytes) const {
    const uintptr_t a = (uintptr_t)p;
    auto it = live.upper_bound(a);
    if (it != live.begin()) {
      --it;
      if (a >= it->first && a + bytes <= it->first + it->second) return true;
    }
    for (const auto& kv : ext)
      if (a >= kv.first && a + bytes <= kv.first + kv.second) return true;
    return false;
  }
};

struct Buf {
  std::shared_ptr<Pool> pool;
  void* p = nullptr;
  size_t c = 0;
  bool ext = false;  // caller-owned range: registered, never freed
  Buf(std::shared_ptr<Pool> pl, size_t bytes) : pool(std::move(pl)) {
    p = pool->get(bytes, c);
    pool->live[(uintptr_t)p] = bytes;
  }
  Buf(std::shared_ptr<Pool> pl, void* extp, size_t bytes) : pool(std::move(pl)), p(extp), c(bytes), ext(true) {
    pool->ext.emplace((uintptr_t)p, bytes);
  }
  ~Buf() {
    if (ext) {
      auto r = pool->ext.equal_range((uintptr_t)p);
      for (auto it = r.first; it != r.second; ++it)
        if (it->second == c) {
          pool->ext.erase(it);
          break;
        }
    } else if (p) {
      pool->live.erase((uintptr_t)p);
      pool->put(p, c);
    }
  }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
};
using BufP = std::shared_ptr<Buf>;

}  // namespace qtt

using qtt::cplx;

namespace qtt {
// a NaN or Inf met in a norm or residual (QTT_ENAN at the ABI)
struct nan_error : std::runtime_error {
  using std::runtime_error::runtime_error;
};
}  // namespace qtt

struct qtt_tensor {
  int kind = 0;  // 0 train, 1 operator, 2 Green operator (factored)
  int L = 0, B = 1;
  std::vector<int> dout, din, r;
  std::vector<char> diag;
  std::vector<cplx*> core, coreR;
  std::vector<qtt::BufP> mem;
  // operators: number of instances stacked per core (a batch of
  // structures), each padded to the common ranks; train batch element b
  // uses instance b / (B / opb)
  int opb = 1;
  // Green operator factors (scheme: QTT_SCHEME_*); the Green step combines
  // q = inv_mu0 u - c p
  std::shared_ptr<qtt_tensor> gU, gS, gP, gE, adj;
  double inv_mu0 = 0.0, c = 0.0;
  int scheme = 0;
  // per-structure Green scalars (device arrays over the train batch) when
  // one factor set serves several reference media
  std::shared_ptr<qtt::Buf> inv_mu0_b, c_b;
  int nbatch_scalars = 0;
  std::shared_ptr<qtt::Pool> pool;

  long celems(int k) const {  // per batch element
    if (kind == 0) return (long)r[k] * dout[k] * r[k + 1];
    if (diag[k]) return (long)r[k] * dout[k] * r[k + 1];
    return (long)r[k] * din[k] * dout[k] * r[k + 1];
  }
};

struct qtt_stat_rec {
  int fam;
  hipEvent_t a, b;  // event pair, or null when the launch recorded a span
  double flops, bytes;
  int slot;         // span slot of the launch (-1: event pair)
};

struct qtt_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  std::shared_ptr<qtt::Pool> pool;
  uint64_t sketch_counter = 0;
  // contractions of a product run in FP32 on the matrix cores while set
  // (rounding, norms and averages always run in FP64)
  bool gemm_fp32 = false;
  // the same with split-BF16 operands and FP32 accumulation
  bool gemm_bf16 = false;
  // statistics family of the next GEMMs when >= 0 (QTT_K_CONTRACT for the
  // operator x train contractions), else by kernel path
  int gemm_family = -1;
  std::map<std::pair<int, int>, std::shared_ptr<qtt_tensor>> ident;  // identity operator per (n, control dim)
  // SFFT and Green factors per (n, delta): shared by every problem of that
  // grid size (the factors do not depend on the reference medium)
  std::map<std::pair<int, double>, std::shared_ptr<qtt_tensor>> sfft_cache;
  std::map<std::tuple<int, double, int>, std::shared_ptr<qtt_tensor>> green_cache;  // (n, delta, scheme)
  // kernel statistics (HIP events around every stats_stride-th launch;
  // flops and bytes of every launch are counted as well)
  bool stats_on = false;
  int stats_stride = 1;
  unsigned long long stats_tick = 0;
  std::vector<qtt_stat_rec> pending;
  std::vector<hipEvent_t> evfree;
  // span slots of the timed matrix-core launches (device {start, end}
  // pairs of real-time counter ticks at span_hz)
  static constexpr int SPAN_SLOTS = 16384;
  unsigned long long* span = nullptr;
  int span_used = 0;
  double span_hz = 0.0;
  long long st_calls[QTT_K_COUNT] = {0};
  double st_secs[QTT_K_COUNT] = {0}, st_flops[QTT_K_COUNT] = {0}, st_bytes[QTT_K_COUNT] = {0};
  long long st_all_calls[QTT_K_COUNT] = {0};
  double st_all_flops[QTT_K_COUNT] = {0}, st_all_bytes[QTT_K_COUNT] = {0};
  // contexts of the concurrent load-case groups (own stream and pool); a
  // sub-context reads the parent's operators
  const qtt_ctx* parent = nullptr;
  std::vector<std::unique_ptr<qtt_ctx>> subs;
  // every context (a group's sub-context too) drains and releases its own
  // stream last, after its sub-contexts, events and span slots
  ~qtt_ctx() {
    subs.clear();
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto& r : pending) {
      if (r.a) (void)hipEventDestroy(r.a);
      if (r.b) (void)hipEventDestroy(r.b);
    }
    for (auto e : evfree) (void)hipEventDestroy(e);
    if (span) (void)hipFree(span);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace qtt {

using TT = qtt_tensor;
using TTP = std::shared_ptr<qtt_tensor>;

static inline cplx C1() { return make_double2(1.0, 0.0); }
static inline cplx C0() { return make_double2(0.0, 0.0); }
static inline cplx CR(double a) { return make_double2(a, 0.0); }

struct Ctx {
  qtt_ctx* c;
  // statistics bracket around one launch
  hipEvent_t ev() const {
    if (!c->evfree.empty()) {
      hipEvent_t e = c->evfree.back();
      c->evfree.pop_back();
      return e;
    }
    hipEvent_t e;
    check(hipEventCreate(&e), "event create");
    return e;
  }
  // t0 before a launch, t1 after it: a null handle when statistics are
  // off, the untimed marker for launches between samples
  static hipEvent_t untimed() { static int tag; return reinterpret_cast<hipEvent_t>(&tag); }
  hipEvent_t t0() const {
    if (!c->stats_on) return nullptr;
    if (c->stats_tick++ % (unsigned long long)c->stats_stride != 0) return untimed();
    hipEvent_t e = ev();
    check(hipEventRecord(e, c->stream), "event record");
    return e;
  }
  void t1(hipEvent_t a, int fam, double flops, double bytes) const {
    if (!a) return;
    c->st_all_calls[fam] += 1;
    c->st_all_flops[fam] += flops;
    c->st_all_bytes[fam] += bytes;
    if (a == untimed()) return;
    hipEvent_t e = ev();
    check(hipEventRecord(e, c->stream), "event record");
    c->pending.push_back({fam, a, e, flops, bytes, -1});
  }
  // a matrix-core launch timed by its own span (first workgroup start to
  // last workgroup end on the real-time counter, written by the kernel):
  // k0 hands out the span pair of a sampled launch (null between samples,
  // slot -1) and returns whether statistics are on; k1 books the launch
  bool k0(unsigned long long*& span, int& slot) const;
  void k1(bool on, int slot, hipEvent_t a, hipEvent_t b, int fam, double flops, double bytes) const {
    if (!on) return;
    c->st_all_calls[fam] += 1;
    c->st_all_flops[fam] += flops;
    c->st_all_bytes[fam] += bytes;
    if (slot >= 0 || a) c->pending.push_back({fam, a, b, flops, bytes, slot});
  }
  hipStream_t s() const { return c->stream; }
  BufP buf(size_t elems) const { return std::make_shared<Buf>(c->pool, std::max<size_t>(elems, 1) * sizeof(cplx)); }
  BufP bufd(size_t n) const { return std::make_shared<Buf>(c->pool, std::max<size_t>(n, 1) * sizeof(double)); }
  void sync() const { check(hipStreamSynchronize(c->stream), "stream sync"); }
};

// Host-side bounds check: the elements base[0..last] (in units of `esz`
// bytes) must lie inside one live device allocation of this context.
static void need(const Ctx& X, const void* base, long last, const char* what, size_t esz = sizeof(cplx)) {
  if (last < 0) return;
  const size_t bytes = (size_t)(last + 1) * esz;
  if (X.c->pool->contains(base, bytes)) return;
  // a sub-context also reads the parent's (idle, read-only) operators, and
  // the parent reads its (idle) sub-contexts' results when it merges them
  if (X.c->parent && X.c->parent->pool->contains(base, bytes)) return;
  for (const auto& sc : X.c->subs)
    if (sc->pool->contains(base, bytes)) return;
  throw std::logic_error(std::string("device operand out of bounds: ") + what);
}
static long span2(long rows, long cols, long rs, long cs) {
  return (rows - 1) * rs + (cols - 1) * cs;
}
// batch layout of a GEMM call: up to three levels (see GemmArgs)
struct Bat {
  int nb1 = 1;
  long sA1 = 0, sB1 = 0, sC1 = 0;
  int nb2 = 1;
  long sA2 = 0, sB2 = 0, sC2 = 0;
  int nb3 = 1;
  long sA3 = 0, sB3 = 0, sC3 = 0;
};
static long spanb(const Bat& t, int w) {
  const long s1 = w == 0 ? t.sA1 : (w == 1 ? t.sB1 : t.sC1);
  const long s2 = w == 0 ? t.sA2 : (w == 1 ? t.sB2 : t.sC2);
  const long s3 = w == 0 ? t.sA3 : (w == 1 ? t.sB3 : t.sC3);
  return (t.nb1 - 1) * s1 + (t.nb2 - 1) * s2 + (t.nb3 - 1) * s3;
}

static void GB(const Ctx& X, int M, int N, int K, int opA, const cplx* A, long lda, int opB,
               const cplx* B, long ldb, cplx* Cm, long ldc, const Bat& t,
               cplx alpha = make_double2(1.0, 0.0), cplx beta = make_double2(0.0, 0.0)) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K; g.opA = opA; g.opB = opB;
  g.A = A; g.lda = lda; g.sA1 = t.sA1; g.sA2 = t.sA2; g.sA3 = t.sA3;
  g.B = B; g.ldb = ldb; g.sB1 = t.sB1; g.sB2 = t.sB2; g.sB3 = t.sB3;
  g.C = Cm; g.ldc = ldc; g.sC1 = t.sC1; g.sC2 = t.sC2; g.sC3 = t.sC3;
  g.nb1 = t.nb1; g.nb2 = t.nb2; g.nb3 = t.nb3; g.alpha = alpha; g.beta = beta;
  if (M > 0 && N > 0 && K > 0) {
    need(X, A, (opA == OP_N ? span2(M, K, lda, 1) : span2(K, M, lda, 1)) + spanb(t, 0), "gemm A");
    need(X, B, (opB == OP_N ? span2(K, N, ldb, 1) : span2(N, K, ldb, 1)) + spanb(t, 1), "gemm B");
    need(X, Cm, span2(M, N, ldc, 1) + spanb(t, 2), "gemm C");
  }
  if (K == 0) throw std::logic_error("gemm with empty contraction");
  const double nb = (double)t.nb1 * t.nb2 * t.nb3;
  BufP ws;
  g.fp32 = X.c->gemm_fp32;
  g.bf16x3 = X.c->gemm_bf16;
  const int ks = gemm_ksplit(M, N, K, (long)nb, g.fp32 || g.bf16x3);
  if (ks > 1) {
    ws = X.buf(gemm_ws_elems(g, ks));
    g.ws = (cplx*)ws->p;
    g.ksplit = ks;
  }
  if (gemm_nbatch(g) > 65535) throw std::runtime_error("gemm: batch too large");
  // the statistics bracket the product kernel alone; the split-K sum of
  // slices (an elementwise pass) is counted with the other helpers
  int slot = -1;
  const bool on = X.k0(g.span, slot);
  int ks_used = 1;
  const bool mc = gemm_mfma_main(g, X.s(), ks_used);
  hipEvent_t ka = nullptr, kb = nullptr;
  if (!mc) {
    // the vector kernel (no span) between stream-position events; the
    // span slot stays unused
    if (slot >= 0) {
      ka = X.ev();
      check(hipEventRecord(ka, X.s()), "event record");
    }
    gemm_vector(g, X.s());
    if (slot >= 0) {
      kb = X.ev();
      check(hipEventRecord(kb, X.s()), "event record");
    }
    slot = -1;
  }
  const int fam = X.c->gemm_family >= 0 ? X.c->gemm_family
                                         : (mc ? (g.bf16x3 ? QTT_K_MFMA_BF16 : (g.fp32 ? QTT_K_MFMA32 : QTT_K_MFMA))
                                               : QTT_K_GEMM);
  X.k1(on, slot, ka, kb, fam, 8.0 * M * N * K * nb,
       16.0 * ((double)M * K + (double)K * N + (beta.x != 0.0 || beta.y != 0.0 ? 2.0 : 1.0) * M * N) * nb);
  if (ks_used > 1) {
    hipEvent_t e2 = X.t0();
    gemm_mfma_reduce(g, ks_used, X.s());
    X.t1(e2, QTT_K_OTHER, 0.0, 16.0 * ((double)ks_used + 1.0 + (beta.x != 0.0 || beta.y != 0.0 ? 1.0 : 0.0)) * M * N * nb);
  }
}

static void G(const Ctx& X, int M, int N, int K, int opA, const cplx* A, long lda, int opB,
              const cplx* B, long ldb, cplx* Cm, long ldc, int nb1 = 1, long sA1 = 0,
              long sB1 = 0, long sC1 = 0, int nb2 = 1, long sA2 = 0, long sB2 = 0,
              long sC2 = 0, cplx alpha = make_double2(1.0, 0.0),
              cplx beta = make_double2(0.0, 0.0)) {
  Bat t;
  t.nb1 = nb1; t.sA1 = sA1; t.sB1 = sB1; t.sC1 = sC1;
  t.nb2 = nb2; t.sA2 = sA2; t.sB2 = sB2; t.sC2 = sC2;
  GB(X, M, N, K, opA, A, lda, opB, B, ldb, Cm, ldc, t, alpha, beta);
}

static double qr_flops(int m, int n, bool q) {
  const double a = std::max(m, n), b = std::min(m, n);
  const double f = 4.0 * (2.0 * a * b * b - 2.0 / 3.0 * b * b * b);
  return q ? 2.0 * f : f;
}


// checked launchers: every device range a kernel touches is verified on the
// host against the live allocations before the launch
static void ck_orth(const Ctx& X, int B, int m, int n, MatView A, MatOut Q, cplx* ws, hipStream_t s,
                    bool drop) {
  need(X, A.base, span2(m, n, A.rs, A.cs) + (B - 1) * A.sb, "orth A");
  need(X, Q.base, span2(m, n, Q.rs, Q.cs) + (B - 1) * Q.sb, "orth Q");
  need(X, ws, (long)orth_split_ws(B, m, n) - 1, "orth ws");
  hipEvent_t e = X.t0();
  if (!orth_split(B, m, n, A, Q, ws, s, drop)) throw std::logic_error("orth: shape not covered");
  // counted as the Householder QR with Q that produces the same basis
  X.t1(e, QTT_K_QR, B * qr_flops(m, n, true), 16.0 * B * 2.0 * m * n);
}
static void ck_qr(const Ctx& X, int B, int m, int n, MatView A, MatOut R, MatOut Q, cplx* ws,
                  hipStream_t s) {
  const int k = std::min(m, n);
  need(X, A.base, span2(m, n, A.rs, A.cs) + (B - 1) * A.sb, "qr A");
  need(X, R.base, span2(k, n, R.rs, R.cs) + (B - 1) * R.sb, "qr R");
  if (Q.base) need(X, Q.base, span2(m, k, Q.rs, Q.cs) + (B - 1) * Q.sb, "qr Q");
  need(X, ws, (long)qr_ws(B, m, n) - 1, "qr ws");
  hipEvent_t e = X.t0();
  qr(B, m, n, A, R, Q, ws, s);
  X.t1(e, QTT_K_QR, B * qr_flops(m, n, Q.base != nullptr), 16.0 * B * ((double)m * n + (double)k * n + (Q.base ? (double)m * k : 0.0)));
}
static void ck_svd(const Ctx& X, int B, int m, int n, MatView A, MatOut U, double* S, MatOut V,
                   cplx* ws, hipStream_t s) {
  need(X, A.base, span2(m, n, A.rs, A.cs) + (B - 1) * A.sb, "svd A");
  need(X, U.base, span2(m, n, U.rs, U.cs) + (B - 1) * U.sb, "svd U");
  need(X, V.base, span2(n, n, V.rs, V.cs) + (B - 1) * V.sb, "svd V");
  need(X, S, (long)B * n - 1, "svd S", sizeof(double));
  need(X, ws, (long)svd_ws(B, m, n) - 1, "svd ws");
  hipEvent_t e = X.t0();
  svd(B, m, n, A, U, S, V, ws, s);
  X.t1(e, QTT_K_JACOBI, B * 4.0 * 22.0 * (double)m * n * n, 16.0 * B * (2.0 * m * n + (double)n * n));
}
static void ck_copy2d(const Ctx& X, int B, int rows, int cols, MatView in, MatOut out, cplx a,
                      hipStream_t s, const double* bscale = nullptr) {
  if (rows <= 0 || cols <= 0 || B <= 0) return;
  need(X, in.base, span2(rows, cols, in.rs, in.cs) + (B - 1) * in.sb, "copy in");
  need(X, out.base, span2(rows, cols, out.rs, out.cs) + (B - 1) * out.sb, "copy out");
  if (bscale) need(X, bscale, B - 1, "copy scale", sizeof(double));
  copy2d(B, rows, cols, in, out, a, s, bscale);
}
static void ck_conj_transpose(const Ctx& X, int B, int rows, int keep, MatView in, MatOut out,
                              hipStream_t s) {
  if (rows <= 0 || keep <= 0 || B <= 0) return;
  need(X, in.base, span2(rows, keep, in.rs, in.cs) + (B - 1) * in.sb, "ctrans in");
  need(X, out.base, span2(keep, rows, out.rs, out.cs) + (B - 1) * out.sb, "ctrans out");
  conj_transpose(B, rows, keep, in, out, s);
}
static void ck_scale_cols(const Ctx& X, int B, int rows, int cols, long ld, long sb, cplx* x,
                          const double* S, long sS, hipStream_t s) {
  if (rows <= 0 || cols <= 0 || B <= 0) return;
  need(X, x, span2(rows, cols, ld, 1) + (B - 1) * sb, "scale x");
  need(X, S, (long)(B - 1) * sS + cols - 1, "scale S", sizeof(double));
  scale_cols(B, rows, cols, ld, sb, x, S, sS, s);
}
static void ck_fill(const Ctx& X, cplx* p, size_t count, cplx v, hipStream_t s) {
  if (count == 0) return;
  need(X, p, (long)count - 1, "fill");
  fill(p, count, v, s);
}
static void ck_batch_norm(const Ctx& X, int B, long len, long stride, const cplx* x, double* out,
                          hipStream_t s) {
  need(X, x, (long)(B - 1) * stride + len - 1, "norm x");
  need(X, out, B - 1, "norm out", sizeof(double));
  batch_norm(B, len, stride, x, out, s);
}
static void ck_sum_middle(const Ctx& X, int B, int outer, int np, int inner, const cplx* in,
                          cplx* out, cplx w, hipStream_t s) {
  need(X, in, (long)B * outer * np * inner - 1, "sum in");
  need(X, out, (long)B * outer * inner - 1, "sum out");
  sum_middle(B, outer, np, inner, in, out, w, s);
}

// allocate a train with given dims and ranks (batch B)
static TTP new_tt(const Ctx& X, int L, int B, const std::vector<int>& dims,
                  const std::vector<int>& ranks) {
  auto t = std::make_shared<TT>();
  t->kind = 0; t->L = L; t->B = B; t->dout = dims; t->din = dims; t->r = ranks;
  t->diag.assign(L, 0);
  t->pool = X.c->pool;
  t->core.resize(L);
  for (int k = 0; k < L; ++k) {
    auto b = X.buf((size_t)B * t->celems(k));
    t->core[k] = (cplx*)b->p;
    t->mem.push_back(b);
  }
  return t;
}

static void set_core(const Ctx& X, TT& t, int k, int r0, int r1, BufP b) {
  t.r[k] = r0;
  t.r[k + 1] = r1;
  t.core[k] = (cplx*)b->p;
  t.mem.push_back(b);
}

static int sat_mul(long a, long b) {
  const long v = a * b;
  return v > (1L << 30) ? (1 << 30) : (int)v;
}

// ---------------------------------------------------------------------------
// truncation sweep (right to left) of a left-orthogonal train
// ---------------------------------------------------------------------------
static int keep_rank(const double* s, int k, double thr, int cap) {
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

struct RoundStats {
  std::vector<double> disc2;  // per batch: sum of discarded sigma^2
  std::vector<double> norm;   // per batch
  double rel_max() const {
    double m = 0.0;
    for (size_t b = 0; b < disc2.size(); ++b)
      if (norm[b] > 0) m = std::max(m, std::sqrt(disc2[b]) / norm[b]);
    return m;
  }
};

// Choose per-batch ranks from singular values S (host, B x kk), zero the
// padded ones, return the common rank; accumulates discarded mass.
static int choose_rank(std::vector<double>& S, int B, int kk, const std::vector<double>& thr, int cap,
                       std::vector<double>& disc2) {
  int rmax = 1;
  std::vector<int> rb(B);
  for (int b = 0; b < B; ++b) {
    rb[b] = keep_rank(&S[(size_t)b * kk], kk, thr[b], cap);
    rmax = std::max(rmax, rb[b]);
  }
  for (int b = 0; b < B; ++b) {
    for (int j = rb[b]; j < kk; ++j) disc2[b] += S[(size_t)b * kk + j] * S[(size_t)b * kk + j];
    for (int j = rb[b]; j < rmax; ++j) S[(size_t)b * kk + j] = 0.0;
  }
  return rmax;
}

// One-sided Jacobi of B square n x n matrices (n <= 320): the LDS kernel
// up to 96, the LDS + workspace kernel beyond.
static void jacobi_any(const Ctx& X, int B, int n, MatView A, MatOut U, double* S) {
  need(X, A.base, span2(n, n, A.rs, A.cs) + (long)(B - 1) * A.sb, "jac in");
  need(X, U.base, span2(n, n, U.rs, U.cs) + (long)(B - 1) * U.sb, "jac U");
  need(X, S, (long)B * n - 1, "jac S", sizeof(double));
  hipEvent_t e = X.t0();
  bool ok;
  if (n <= 96) {
    ok = jacobi_square(B, n, A, U, S, X.s());
  } else {
    auto ws = X.buf(jacobi_ws(B, n));
    ok = jacobi_big(B, n, A, U, S, (cplx*)ws->p, X.s());
  }
  if (!ok) throw std::logic_error("jacobi size");
  X.t1(e, QTT_K_JACOBI, B * 4.0 * 22.0 * (double)n * n * n, 16.0 * B * 2.0 * n * n);
}

static void truncate_rl(const Ctx& X, TT& y, double delta, int cap, RoundStats* st) {
  const int L = y.L, B = y.B;
  std::vector<double> nrm(B);
  {
    auto nb = X.bufd(B);
    ck_batch_norm(X, B, y.celems(L - 1), y.celems(L - 1), y.core[L - 1], (double*)nb->p, X.s());
    check(hipMemcpyAsync(nrm.data(), nb->p, B * sizeof(double), hipMemcpyDeviceToHost, X.s()), "norm d2h");
    X.sync();
  }
  for (int b = 0; b < B; ++b)
    if (!std::isfinite(nrm[b])) throw nan_error("NaN/Inf in the norm of a train being rounded");
  std::vector<double> thr(B), disc2(B, 0.0);
  for (int b = 0; b < B; ++b) thr[b] = delta / std::sqrt((double)std::max(L - 1, 1)) * nrm[b];
  // host arrays of the per-bond uploads stay alive until the sweep's
  // single final synchronisation (no wait at the end of every bond); the
  // guard, destroyed first, drains the stream on every exit
  std::vector<std::vector<double>> hold;
  struct Drain {
    hipStream_t s;
    ~Drain() { (void)hipStreamSynchronize(s); }
  } drain{X.s()};
  for (int k = L - 1; k >= 1; --k) {
    const int p = y.r[k], q = y.dout[k] * y.r[k + 1];
    const int kk = std::min(p, q);
    const int rows = y.r[k - 1] * y.dout[k - 1];
    const long msz = (long)p * q;
    if (kk <= 160 && std::max(p, q) <= 320) {
      // small square factor: R of the tall orientation, Jacobi on it in LDS
      auto R = X.buf((size_t)B * kk * kk);
      auto U = X.buf((size_t)B * kk * kk);
      auto Sd = X.bufd((size_t)B * kk);
      BufP Qb;
      if (p <= q) {
        auto ws = X.buf(qr_ws(B, q, p));
        ck_qr(X, B, q, p, MatView{y.core[k], 1, (long)q, msz, 1},
              MatOut{(cplx*)R->p, (long)kk, 1, (long)kk * kk}, MatOut{nullptr, 0, 0, 0}, (cplx*)ws->p, X.s());
        // Jacobi on R^H: left singular vectors of M
        jacobi_any(X, B, kk, MatView{(cplx*)R->p, 1, (long)kk, (long)kk * kk, 1},
                   MatOut{(cplx*)U->p, (long)kk, 1, (long)kk * kk}, (double*)Sd->p);
      } else {
        Qb = X.buf((size_t)B * p * q);
        auto ws = X.buf(qr_ws(B, p, q));
        ck_qr(X, B, p, q, MatView{y.core[k], (long)q, 1, msz, 0},
              MatOut{(cplx*)R->p, (long)kk, 1, (long)kk * kk}, MatOut{(cplx*)Qb->p, (long)q, 1, msz},
              (cplx*)ws->p, X.s());
        jacobi_any(X, B, kk, MatView{(cplx*)R->p, (long)kk, 1, (long)kk * kk, 0},
                   MatOut{(cplx*)U->p, (long)kk, 1, (long)kk * kk}, (double*)Sd->p);
      }
      std::vector<double> S((size_t)B * kk);
      check(hipMemcpyAsync(S.data(), Sd->p, S.size() * sizeof(double), hipMemcpyDeviceToHost, X.s()), "S d2h");
      X.sync();
      const int rmax = choose_rank(S, B, kk, thr, cap, disc2);
      std::vector<double> SI(S.size());
      for (size_t e = 0; e < S.size(); ++e) SI[e] = S[e] > 0.0 ? 1.0 / S[e] : 0.0;
      auto Sdev = X.bufd(S.size());
      auto SIdev = X.bufd(S.size());
      check(hipMemcpyAsync(Sdev->p, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice, X.s()), "S h2d");
      check(hipMemcpyAsync(SIdev->p, SI.data(), SI.size() * sizeof(double), hipMemcpyHostToDevice, X.s()), "S h2d");
      auto U2 = X.buf((size_t)B * kk * kk);
      ck_copy2d(X, B, kk, kk, MatView{(cplx*)U->p, (long)kk, 1, (long)kk * kk, 0},
                MatOut{(cplx*)U2->p, (long)kk, 1, (long)kk * kk}, C1(), X.s());
      ck_scale_cols(X, B, kk, rmax, kk, (long)kk * kk, (cplx*)U->p, (double*)SIdev->p, kk, X.s());
      ck_scale_cols(X, B, kk, rmax, kk, (long)kk * kk, (cplx*)U2->p, (double*)Sdev->p, kk, X.s());
      auto nk = X.buf((size_t)B * rmax * q);
      auto nk1 = X.buf((size_t)B * rows * rmax);
      if (p <= q) {
        // new core = (U S^-1)^H M ; absorbed = U S
        G(X, rmax, q, p, OP_C, (cplx*)U->p, kk, OP_N, y.core[k], q, (cplx*)nk->p, q, B,
          (long)kk * kk, msz, (long)rmax * q);
        G(X, rows, rmax, p, OP_N, y.core[k - 1], p, OP_N, (cplx*)U2->p, kk, (cplx*)nk1->p, rmax, B,
          (long)rows * p, (long)kk * kk, (long)rows * rmax);
      } else {
        // M = Q R, R = U S W^H: new core = (U S^-1)^H R ; absorbed = Q U S
        G(X, rmax, q, q, OP_C, (cplx*)U->p, kk, OP_N, (cplx*)R->p, kk, (cplx*)nk->p, q, B,
          (long)kk * kk, (long)kk * kk, (long)rmax * q);
        auto T = X.buf((size_t)B * p * rmax);
        G(X, p, rmax, q, OP_N, (cplx*)Qb->p, q, OP_N, (cplx*)U2->p, kk, (cplx*)T->p, rmax, B, msz,
          (long)kk * kk, (long)p * rmax);
        G(X, rows, rmax, p, OP_N, y.core[k - 1], p, OP_N, (cplx*)T->p, rmax, (cplx*)nk1->p, rmax, B,
          (long)rows * p, (long)p * rmax, (long)rows * rmax);
      }
      // Row j of W = (U S^-1)^H M carries an error of about
      // eps * sigma_0 / sigma_j, so with kept singular values far apart the
      // rows of the new core are no longer orthonormal (the later bonds'
      // thresholds and the discarded mass assume they are).  Then W is
      // split as W = R^H Q^H (QR of W^H): the core becomes Q^H, exactly
      // orthonormal, and R^H moves into the absorbed factor, so the
      // product (U S) W is unchanged.
      double spread = 1.0;
      for (int b = 0; b < B; ++b) {
        const double s0 = S[(size_t)b * kk];
        for (int j = 0; j < rmax; ++j) {
          const double sj = S[(size_t)b * kk + j];
          if (sj > 0.0) spread = std::max(spread, s0 / sj);
        }
      }
      if (spread > 1e6) {
        auto Qw = X.buf((size_t)B * q * rmax);
        auto Rw = X.buf((size_t)B * rmax * rmax);
        auto ws = X.buf(qr_ws(B, q, rmax));
        ck_qr(X, B, q, rmax, MatView{(cplx*)nk->p, 1, (long)q, (long)rmax * q, 1},
              MatOut{(cplx*)Rw->p, (long)rmax, 1, (long)rmax * rmax},
              MatOut{(cplx*)Qw->p, (long)rmax, 1, (long)q * rmax}, (cplx*)ws->p, X.s());
        ck_conj_transpose(X, B, q, rmax, MatView{(cplx*)Qw->p, (long)rmax, 1, (long)q * rmax, 0},
                          MatOut{(cplx*)nk->p, (long)q, 1, (long)rmax * q}, X.s());
        auto nk2 = X.buf((size_t)B * rows * rmax);
        G(X, rows, rmax, rmax, OP_N, (cplx*)nk1->p, rmax, OP_C, (cplx*)Rw->p, rmax, (cplx*)nk2->p, rmax,
          B, (long)rows * rmax, (long)rmax * rmax, (long)rows * rmax);
        nk1 = nk2;
      }
      hold.push_back(std::move(S));
      hold.push_back(std::move(SI));
      set_core(X, y, k, rmax, y.r[k + 1], nk);
      set_core(X, y, k - 1, y.r[k - 1], rmax, nk1);
      continue;
    }
    auto LV = X.buf((size_t)B * p * kk);
    auto RV = X.buf((size_t)B * q * kk);
    auto Sd = X.bufd((size_t)B * kk);
    cplx* lv = (cplx*)LV->p;
    cplx* rv = (cplx*)RV->p;
    double* sd = (double*)Sd->p;
    if (p <= q) {
      auto ws = X.buf(svd_ws(B, q, p));
      ck_svd(X, B, q, p, MatView{y.core[k], 1, (long)q, msz, 1}, MatOut{rv, (long)kk, 1, (long)q * kk}, sd,
             MatOut{lv, (long)kk, 1, (long)p * kk}, (cplx*)ws->p, X.s());
    } else {
      auto ws = X.buf(svd_ws(B, p, q));
      ck_svd(X, B, p, q, MatView{y.core[k], (long)q, 1, msz, 0}, MatOut{lv, (long)kk, 1, (long)p * kk}, sd,
             MatOut{rv, (long)kk, 1, (long)q * kk}, (cplx*)ws->p, X.s());
    }
    std::vector<double> S((size_t)B * kk);
    check(hipMemcpyAsync(S.data(), sd, S.size() * sizeof(double), hipMemcpyDeviceToHost, X.s()), "S d2h");
    X.sync();
    const int rmax = choose_rank(S, B, kk, thr, cap, disc2);
    check(hipMemcpyAsync(sd, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice, X.s()), "S h2d");
    auto nk = X.buf((size_t)B * rmax * q);
    ck_conj_transpose(X, B, q, rmax, MatView{rv, (long)kk, 1, (long)q * kk, 0},
                      MatOut{(cplx*)nk->p, (long)q, 1, (long)rmax * q}, X.s());
    ck_scale_cols(X, B, p, rmax, kk, (long)p * kk, lv, sd, kk, X.s());
    auto nk1 = X.buf((size_t)B * rows * rmax);
    G(X, rows, rmax, p, OP_N, y.core[k - 1], p, OP_N, lv, kk, (cplx*)nk1->p, rmax, B,
      (long)rows * p, (long)p * kk, (long)rows * rmax);
    hold.push_back(std::move(S));
    set_core(X, y, k, rmax, y.r[k + 1], nk);
    set_core(X, y, k - 1, y.r[k - 1], rmax, nk1);
  }
  X.sync();  // the uploads of `hold` have been consumed
  if (st) {
    st->disc2 = disc2;
    st->norm = nrm;
  }
}

// explicit rounding: left-to-right QR sweep, then truncation sweep
static void round_tt(const Ctx& X, TT& x, double delta, int cap, RoundStats* st) {
  const int L = x.L, B = x.B;
  for (int k = 0; k < L - 1; ++k) {
    const int m = x.r[k] * x.dout[k], n = x.r[k + 1];
    const int kq = std::min(m, n);
    auto Q = X.buf((size_t)B * m * kq);
    auto R = X.buf((size_t)B * kq * n);
    auto ws = X.buf(qr_ws(B, m, n));
    ck_qr(X, B, m, n, MatView{x.core[k], (long)n, 1, (long)m * n, 0},
       MatOut{(cplx*)R->p, (long)n, 1, (long)kq * n}, MatOut{(cplx*)Q->p, (long)kq, 1, (long)m * kq},
       (cplx*)ws->p, X.s());
    const int cols = x.dout[k + 1] * x.r[k + 2];
    auto nx = X.buf((size_t)B * kq * cols);
    G(X, kq, cols, n, OP_N, (cplx*)R->p, n, OP_N, x.core[k + 1], cols, (cplx*)nx->p, cols, B,
      (long)kq * n, (long)n * cols, (long)kq * cols);
    set_core(X, x, k, x.r[k], kq, Q);
    set_core(X, x, k + 1, kq, x.r[k + 2], nx);
  }
  truncate_rl(X, x, delta, cap, st);
}

// Frobenius norms via a left-to-right QR sweep that keeps only R factors.
static std::vector<double> tt_norms(const Ctx& X, const TT& x) {
  const int L = x.L, B = x.B;
  BufP cur;  // current (R * core_k)
  const cplx* curp = x.core[0];
  int rows = x.r[0] * x.dout[0];
  for (int k = 0; k < L - 1; ++k) {
    const int m = rows, n = x.r[k + 1];
    const int kq = std::min(m, n);
    auto R = X.buf((size_t)B * kq * n);
    auto ws = X.buf(qr_ws(B, m, n));
    ck_qr(X, B, m, n, MatView{curp, (long)n, 1, (long)m * n, 0},
       MatOut{(cplx*)R->p, (long)n, 1, (long)kq * n}, MatOut{nullptr, 0, 0, 0}, (cplx*)ws->p, X.s());
    const int cols = x.dout[k + 1] * x.r[k + 2];
    auto nx = X.buf((size_t)B * kq * cols);
    G(X, kq, cols, n, OP_N, (cplx*)R->p, n, OP_N, x.core[k + 1], cols, (cplx*)nx->p, cols, B,
      (long)kq * n, (long)n * cols, (long)kq * cols);
    cur = nx;
    curp = (cplx*)nx->p;
    rows = kq * x.dout[k + 1];
  }
  const long len = (long)rows * x.r[L];
  auto nb = X.bufd(B);
  ck_batch_norm(X, B, len, len, curp, (double*)nb->p, X.s());
  std::vector<double> out(B);
  check(hipMemcpyAsync(out.data(), nb->p, B * sizeof(double), hipMemcpyDeviceToHost, X.s()), "norm d2h");
  X.sync();
  for (int b = 0; b < B; ++b)
    if (!std::isfinite(out[b])) throw nan_error("NaN/Inf in a train norm");
  return out;
}

// z = alpha x + beta y (block cores)
// z = alpha x + beta y (block concatenation of the cores); alpha_b, beta_b:
// optional per-batch-element factors (device) multiplying alpha, beta
static TTP axpby(const Ctx& X, double alpha, const TT& x, double beta, const TT& y,
                 const double* alpha_b = nullptr, const double* beta_b = nullptr) {
  if (x.L != y.L || x.B != y.B) throw std::invalid_argument("axpby: shape mismatch");
  const int L = x.L, B = x.B;
  std::vector<int> rz(L + 1);
  rz[0] = 1; rz[L] = 1;
  for (int k = 1; k < L; ++k) rz[k] = x.r[k] + y.r[k];
  auto z = new_tt(X, L, B, x.dout, rz);
  for (int k = 0; k < L; ++k) {
    const int d = x.dout[k];
    const int R0 = rz[k], R1 = rz[k + 1];
    ck_fill(X, z->core[k], (size_t)B * R0 * d * R1, C0(), X.s());
    const int xr0 = x.r[k], xr1 = x.r[k + 1], yr0 = y.r[k], yr1 = y.r[k + 1];
    const long zsb = (long)R0 * d * R1;
    // x block at (0, 0)
    ck_copy2d(X, B, xr0 * d, xr1, MatView{x.core[k], (long)xr1, 1, (long)xr0 * d * xr1, 0},
           MatOut{z->core[k], (long)R1, 1, zsb}, CR(k == 0 ? alpha : 1.0), X.s(),
           k == 0 ? alpha_b : nullptr);
    // y block at row offset (k>0 ? xr0*d : 0), col offset (k<L-1 ? xr1 : 0)
    const long roff = (k > 0) ? (long)xr0 * d : 0;
    const long coff = (k < L - 1) ? xr1 : 0;
    if (k == 0 || k == L - 1) {
      // first core: concatenate columns; last core: stack rows
      ck_copy2d(X, B, yr0 * d, yr1, MatView{y.core[k], (long)yr1, 1, (long)yr0 * d * yr1, 0},
             MatOut{z->core[k] + roff * R1 + coff, (long)R1, 1, zsb}, CR(k == 0 ? beta : 1.0), X.s(),
             k == 0 ? beta_b : nullptr);
      if (k == 0 && L == 1) throw std::invalid_argument("axpby: L == 1");
    } else {
      ck_copy2d(X, B, yr0 * d, yr1, MatView{y.core[k], (long)yr1, 1, (long)yr0 * d * yr1, 0},
             MatOut{z->core[k] + roff * R1 + coff, (long)R1, 1, zsb}, CR(1.0), X.s());
    }
  }
  // the first core: x and y blocks share the single row; the copies above
  // placed y at column offset xr1 with row offset 0 (k = 0), correct.
  // The last core: y rows follow x rows at column 0, correct.
  return z;
}

// ---------------------------------------------------------------------------
// operator application
// ---------------------------------------------------------------------------
struct SketchOpts {
  double delta = 1e-10;
  int cap = 0;
  int oversample = 16;
  bool exact = false;
  uint64_t seed = 0;
  // keep the left-orthogonal sketch result (ranks <= cap + oversample)
  // without the final truncated-SVD sweep: used for intermediate products
  // whose result is immediately sketched again
  bool no_truncate = false;
  // contractions in FP32 (QR, SVD and the truncation stay FP64)
  bool fp32 = false;
  // contractions with split-BF16 operands and FP32 accumulation
  bool bf16 = false;
  // range-finder bases: QTT_ORTH_HOUSEHOLDER, _CHOLQR or _AUTO
  int orth = QTT_ORTH_HOUSEHOLDER;
  // the fixed-point iterate entering this product has a bond rank at the
  // cap (QTT_ORTH_AUTO then takes CholeskyQR2: the sketches are full rank)
  bool saturated = false;
  // QTT_MV_AMEN: the Green step's factor products by the AMEn-adapted
  // product, warm-started from the previous update's results in `amen`
  int matvec = 0;
  struct AmenSlots* amen = nullptr;
};

// reduced-precision contractions (FP32, split-BF16) for the lifetime of
// the scope (restores the previous setting; off() ends it early)
struct Fp32Scope {
  qtt_ctx* c;
  bool prev, prevb;
  Fp32Scope(const Ctx& X, bool on) : c(X.c), prev(X.c->gemm_fp32), prevb(X.c->gemm_bf16) {
    c->gemm_fp32 = on;
    c->gemm_bf16 = false;
  }
  void off() {
    c->gemm_fp32 = prev;
    c->gemm_bf16 = prevb;
  }
  ~Fp32Scope() { off(); }
};

// Contract Mc (B, lt, rho, r) with x_k -> T1 (B, lt, rho, din, r2), then with
// the operator core -> P (B, lt, dout, rho2, r2).
static BufP left_step(const Ctx& X, const TT& A, const TT& x, int k, const cplx* Mc, int lt) {
  const int B = x.B;
  const int rho = A.r[k], rho2 = A.r[k + 1], r = x.r[k], r2 = x.r[k + 1];
  const int din = x.dout[k], dout = A.dout[k];
  auto T1 = X.buf((size_t)B * lt * rho * din * r2);
  G(X, lt * rho, din * r2, r, OP_N, Mc, r, OP_N, x.core[k], (long)din * r2, (cplx*)T1->p,
    (long)din * r2, B, (long)lt * rho * r, (long)r * din * r2, (long)lt * rho * din * r2);
  auto P = X.buf((size_t)B * lt * dout * rho2 * r2);
  // operator instance per group of g train elements (g = B for one instance)
  const int ob = A.opb, g = B / ob;
  if (B % ob) throw std::invalid_argument("train batch not a multiple of the operator instances");
  const long ia = ob > 1 ? A.celems(k) : 0;
  Bat t;
  t.nb1 = ob;
  t.sA1 = ia;
  t.nb2 = g * lt;
  X.c->gemm_family = QTT_K_CONTRACT;
  if (!A.diag[k]) {
    t.sB1 = (long)g * lt * rho * din * r2; t.sC1 = (long)g * lt * dout * rho2 * r2;
    t.sB2 = (long)rho * din * r2; t.sC2 = (long)dout * rho2 * r2;
    GB(X, dout * rho2, r2, rho * din, OP_T, A.core[k], (long)dout * rho2, OP_N, (cplx*)T1->p, r2,
       (cplx*)P->p, r2, t);
  } else {
    const int d = dout;
    t.sB1 = (long)g * lt * rho * d * r2; t.sC1 = (long)g * lt * d * rho2 * r2;
    t.sB2 = (long)rho * d * r2; t.sC2 = (long)d * rho2 * r2;
    t.nb3 = d; t.sA3 = rho2; t.sB3 = r2; t.sC3 = (long)rho2 * r2;
    GB(X, rho2, r2, rho, OP_T, A.core[k], (long)d * rho2, OP_N, (cplx*)T1->p, (long)d * r2,
       (cplx*)P->p, r2, t);
  }
  X.c->gemm_family = -1;
  return P;
}

// Right-to-left step of the sketch (and of the frame interfaces of the
// AMEn product): X1 = x_k W_{k+1} (B, r, din, rho2, l2), then the operator
// core -> X2 (B, r, rho, dout, l2); W2 is (B, rho_{k+1}, r_{k+1}, l2).
static BufP right_contract(const Ctx& X, const TT& A, const TT& x, int k, const cplx* W2, int l2) {
  const int B = x.B;
  const int rho = A.r[k], rho2 = A.r[k + 1], r = x.r[k], r2 = x.r[k + 1];
  const int din = x.dout[k], dout = A.dout[k];
  auto X1 = X.buf((size_t)B * r * din * rho2 * l2);
  G(X, r * din, l2, r2, OP_N, x.core[k], r2, OP_N, W2, l2, (cplx*)X1->p, (long)rho2 * l2, B,
    (long)r * din * r2, (long)rho2 * r2 * l2, (long)r * din * rho2 * l2, rho2, 0,
    (long)r2 * l2, l2);
  auto X2 = X.buf((size_t)B * r * rho * dout * l2);
  const int ob = A.opb, g = B / ob;
  const long ia = ob > 1 ? A.celems(k) : 0;
  Bat t;
  t.nb1 = ob;
  t.sA1 = ia;
  t.nb2 = g * r;
  X.c->gemm_family = QTT_K_CONTRACT;
  if (!A.diag[k]) {
    t.sB1 = (long)g * r * din * rho2 * l2; t.sC1 = (long)g * r * rho * dout * l2;
    t.sB2 = (long)din * rho2 * l2; t.sC2 = (long)rho * dout * l2;
    GB(X, rho * dout, l2, din * rho2, OP_N, A.coreR[k], (long)din * rho2, OP_N, (cplx*)X1->p, l2,
       (cplx*)X2->p, l2, t);
  } else {
    const int d = dout;
    t.sB1 = (long)g * r * d * rho2 * l2; t.sC1 = (long)g * r * rho * d * l2;
    t.sB2 = (long)d * rho2 * l2; t.sC2 = (long)rho * d * l2;
    t.nb3 = d; t.sA3 = rho2; t.sB3 = (long)rho2 * l2; t.sC3 = l2;
    GB(X, rho, l2, rho2, OP_N, A.core[k], (long)d * rho2, OP_N, (cplx*)X1->p, l2, (cplx*)X2->p,
       (long)d * l2, t);
  }
  X.c->gemm_family = -1;
  return X2;
}

// W (B, rho, r, l) = X2 (B, r, rho, dout, l2) contracted over (dout, l2)
// with a core Om (l, dout, l2): op OP_T takes Om itself (a Gaussian test
// core, shared by the batch: oms = 0), OP_C its conjugate (a frame core,
// one per batch element: oms = its size).
static void right_project(const Ctx& X, int B, int rho, int r, int dout, int l2, const cplx* X2, int op,
                          const cplx* Om, long oms, int l, cplx* W) {
  if (rho >= r) {
    // rows a of X2[b][c] against Om: one product per (b, c)
    G(X, rho, l, dout * l2, OP_N, X2, (long)dout * l2, op, Om, (long)dout * l2, W, (long)r * l, B,
      (long)r * rho * dout * l2, oms, (long)rho * r * l, r, (long)rho * dout * l2, 0, l);
  } else {
    // rows c (stride rho dout l2) against Om: one product per (b, a), the
    // longer of the two row counts on the matrix-core M side
    G(X, r, l, dout * l2, OP_N, X2, (long)rho * dout * l2, op, Om, (long)dout * l2, W, (long)l, B,
      (long)r * rho * dout * l2, oms, (long)rho * r * l, rho, (long)dout * l2, 0, (long)r * l);
  }
}

static TTP sketch_apply(const Ctx& X, const TT& A, const TT& x, const SketchOpts& o,
                        RoundStats* st) {
  const int L = x.L, B = x.B;
  if (A.L != L) throw std::invalid_argument("operator and train differ in length");
  if (B % A.opb) throw std::invalid_argument("train batch not a multiple of the operator instances");
  for (int k = 0; k < L; ++k)
    if (A.din[k] != x.dout[k]) throw std::invalid_argument("operator input dim mismatch");
  // FP32 (o.fp32) is used only for contractions whose operands are well
  // conditioned: the operator x train step (T1) and the projection onto the
  // orthonormal QR basis (Q^H P).  The Gaussian tensor-train sketches are
  // ill-conditioned (their condition numbers multiply along the train), so
  // the partial sketches W and the sketched unfoldings Y = P W stay FP64.
  const bool f32 = o.fp32 && !o.exact, b16 = o.bf16 && !o.exact;
  Fp32Scope prec(X, false);
  // sketch ranks
  std::vector<int> ell(L + 1, 1);
  std::vector<long> left(L + 1, 1), right(L + 1, 1);
  for (int k = 1; k <= L; ++k) left[k] = std::min<long>(left[k - 1] * A.dout[k - 1], 1L << 30);
  for (int k = L - 1; k >= 0; --k) right[k] = std::min<long>(right[k + 1] * A.dout[k], 1L << 30);
  // Exact mode uses deterministic test matrices: the full right unfolding
  // of the product at the bonds nearest the right end whose right dimension
  // does not exceed the product rank ("dense"), and the identity (no
  // sketch: the left-to-right sweep then QR-factors the product unfolding
  // itself) at every bond further left.
  std::vector<char> dense_w(L + 1, 0), ident_w(L + 1, 0);
  if (o.exact || o.cap <= 0) {
    bool run = true;
    for (int k = L - 1; k >= 1; --k) {
      const long pr = (long)sat_mul(A.r[k], x.r[k]);
      if (run && right[k] <= pr) {
        dense_w[k] = 1;
        ell[k] = (int)right[k];
      } else {
        run = false;
        ident_w[k] = 1;
        ell[k] = (int)pr;
      }
    }
  } else {
    for (int k = 1; k < L; ++k) {
      long e = std::min<long>((long)sat_mul(A.r[k], x.r[k]), std::min(left[k], right[k]));
      e = std::min<long>(e, (long)o.cap + o.oversample);
      ell[k] = (int)std::max<long>(1, e);
    }
  }
  // random test train Omega_k (ell_k, dout_k, ell_{k+1}), k = 1..L-1
  // (drawn in as few launches as the block limit allows)
  std::vector<BufP> Om(L);
  GaussBlocks gb;
  gb.start[0] = 0;
  for (int k = 1; k < L; ++k) {
    if (dense_w[k] || ident_w[k]) continue;
    const size_t cnt = (size_t)ell[k] * A.dout[k] * ell[k + 1];
    Om[k] = X.buf(cnt);
    need(X, Om[k]->p, (long)cnt - 1, "gaussian");
    gb.out[gb.n] = (cplx*)Om[k]->p;
    gb.stream[gb.n] = (uint64_t)k;
    gb.scale[gb.n] = 1.0 / std::sqrt((double)A.dout[k] * ell[k + 1]);
    gb.start[gb.n + 1] = gb.start[gb.n] + (long)cnt;
    if (++gb.n == GAUSS_MULTI_MAX) {
      gaussian_multi(gb, o.seed, X.s());
      gb.n = 0;
    }
  }
  gaussian_multi(gb, o.seed, X.s());
  // right-to-left partial sketches W_k (B, rho_k, r_k, ell_k)
  std::vector<BufP> W(L + 1);
  W[L] = X.buf(B);
  ck_fill(X, (cplx*)W[L]->p, B, C1(), X.s());
  for (int k = L - 1; k >= 1; --k) {
    if (ident_w[k]) break;  // every bond further left is an identity bond
    const int rho = A.r[k], r = x.r[k], dout = A.dout[k];
    const int l2 = ell[k + 1], l = ell[k];
    auto X2 = right_contract(X, A, x, k, (const cplx*)W[k + 1]->p, l2);
    W[k] = X.buf((size_t)B * rho * r * l);
    if (dense_w[k]) {
      // W_k[b][a][c][(i t)] = X2[b][c][a][(i t)]  (l = dout * l2)
      const long m = (long)dout * l2;
      for (int b = 0; b < B; ++b)
        ck_copy2d(X, r, rho, (int)m, MatView{(cplx*)X2->p + (long)b * r * rho * m, m, 1, rho * m, 0},
                  MatOut{(cplx*)W[k]->p + (long)b * rho * r * m, (long)r * m, 1, m}, C1(), X.s());
    } else {
      right_project(X, B, rho, r, dout, l2, (const cplx*)X2->p, OP_T, (const cplx*)Om[k]->p, 0, l,
                    (cplx*)W[k]->p);
    }
  }
  // left-to-right: QR of sketched unfoldings
  std::vector<int> ry(L + 1, 1);
  auto y = std::make_shared<TT>();
  y->kind = 0; y->L = L; y->B = B; y->dout = A.dout; y->din = A.dout; y->r = ry;
  y->diag.assign(L, 0); y->core.resize(L); y->pool = X.c->pool;
  auto Mc = X.buf(B);
  ck_fill(X, (cplx*)Mc->p, B, C1(), X.s());
  int lt = 1;
  for (int k = 0; k < L; ++k) {
    const int rho2 = A.r[k + 1], r2 = x.r[k + 1], dout = A.dout[k];
    X.c->gemm_fp32 = f32;
    X.c->gemm_bf16 = b16;
    auto P = left_step(X, A, x, k, (cplx*)Mc->p, lt);
    X.c->gemm_fp32 = false;
    X.c->gemm_bf16 = false;
    if (k == L - 1) {
      set_core(X, *y, k, lt, 1, P);
      break;
    }
    const int l2 = ell[k + 1];
    const int m = lt * dout, kq = std::min(m, l2);
    BufP Y;
    if (ident_w[k + 1]) {
      Y = P;  // l2 == rho2 * r2: factor the product unfolding itself
    } else {
      Y = X.buf((size_t)B * m * l2);
      G(X, m, l2, rho2 * r2, OP_N, (cplx*)P->p, (long)rho2 * r2, OP_N, (cplx*)W[k + 1]->p, l2,
        (cplx*)Y->p, l2, B, (long)m * rho2 * r2, (long)rho2 * r2 * l2, (long)m * l2);
    }
    auto Q = X.buf((size_t)B * m * kq);
    const MatView yv{(cplx*)Y->p, (long)l2, 1, (long)m * l2, 0};
    const MatOut qv{(cplx*)Q->p, (long)kq, 1, (long)m * kq};
    const bool cq = o.orth == QTT_ORTH_CHOLQR || (o.orth == QTT_ORTH_AUTO && o.saturated);
    if (cq && !o.exact && orth_ok(m, l2)) {
      // only the basis is kept (R is not needed): CholeskyQR2 on the matrix
      // cores, Householder for the matrices it cannot take
      auto ws = X.buf(orth_split_ws(B, m, l2));
      // cap-bound updates (QTT_ORTH_AUTO): dependent columns of the sketch
      // become zero columns of the basis instead of a fallback; the rounding
      // only needs an isometry on the range, and the dropped directions
      // (below 3e-7 relative) lie far under the cap's truncation
      ck_orth(X, B, m, l2, yv, qv, (cplx*)ws->p, X.s(), o.orth == QTT_ORTH_AUTO);
    } else {
      auto R = X.buf((size_t)B * kq * l2);
      auto ws = X.buf(qr_ws(B, m, l2));
      ck_qr(X, B, m, l2, yv, MatOut{(cplx*)R->p, (long)l2, 1, (long)kq * l2}, qv, (cplx*)ws->p, X.s());
    }
    auto Mn = X.buf((size_t)B * kq * rho2 * r2);
    X.c->gemm_fp32 = f32;
    X.c->gemm_bf16 = b16;
    G(X, kq, rho2 * r2, m, OP_C, (cplx*)Q->p, kq, OP_N, (cplx*)P->p, (long)rho2 * r2, (cplx*)Mn->p,
      (long)rho2 * r2, B, (long)m * kq, (long)m * rho2 * r2, (long)kq * rho2 * r2);
    X.c->gemm_fp32 = false;
    X.c->gemm_bf16 = false;
    set_core(X, *y, k, lt, kq, Q);
    Mc = Mn;
    lt = kq;
  }
  prec.off();
  if (o.no_truncate && !o.exact && o.cap > 0) {
    if (st) {
      st->disc2.assign(B, 0.0);
      st->norm.assign(B, 1.0);
    }
    return y;
  }
  truncate_rl(X, *y, o.delta, o.cap, st);
  return y;
}

// Materialised product (ranks multiply).
static TTP apply_full(const Ctx& X, const TT& A, const TT& x) {
  const int L = x.L, B = x.B;
  if (B % A.opb) throw std::invalid_argument("train batch not a multiple of the operator instances");
  std::vector<int> rz(L + 1);
  for (int k = 0; k <= L; ++k) rz[k] = A.r[k] * x.r[k];
  auto z = new_tt(X, L, B, A.dout, rz);
  // one launch for every core (descriptors uploaded with the call)
  std::vector<TtoDesc> d(L);
  long blocks = 0;
  double flops = 0.0, bytes = 0.0;
  for (int k = 0; k < L; ++k) {
    const int rho = A.r[k], din = A.diag[k] ? 0 : A.din[k], dout = A.dout[k], rho2 = A.r[k + 1];
    const int r = x.r[k], r2 = x.r[k + 1];
    const long dx = din > 0 ? din : dout;
    const long total = (long)B * rho * r * dout * rho2 * r2;
    const long ainst = (long)rho * (din > 0 ? din : 1) * dout * rho2;
    // 32-bit offsets inside a core's output, input and operator instance
    if (total >= (1L << 31) || (long)B * r * dx * r2 >= (1L << 31) || ainst >= (1L << 31))
      throw std::invalid_argument("product core too large for one launch");
    need(X, A.core[k], ainst * A.opb - 1, "apply A");
    need(X, x.core[k], (long)B * r * dx * r2 - 1, "apply x");
    need(X, z->core[k], total - 1, "apply Z");
    d[k] = TtoDesc{A.core[k], x.core[k], z->core[k], B, rho, din, dout, rho2, r, r2, total, blocks,
                   A.opb > 1 ? ainst : 0, B / A.opb};
    d[k].f_cols = make_fastdiv((uint32_t)(total / ((long)dout * rho2)));
    d[k].f_r2 = make_fastdiv((uint32_t)r2);
    d[k].f_r = make_fastdiv((uint32_t)r);
    d[k].f_rho = make_fastdiv((uint32_t)rho);
    d[k].f_group = make_fastdiv((uint32_t)(B / A.opb));
    blocks += tto_apply_blocks(total, rho2);
    flops += (double)total * 8.0 * (din > 0 ? din : 1);
    bytes += 16.0 * ((double)rho * (din > 0 ? din : 1) * dout * rho2 + (double)B * r * dx * r2 + (double)total);
  }
  auto dd = X.buf((d.size() * sizeof(TtoDesc) + sizeof(cplx) - 1) / sizeof(cplx));
  check(hipMemcpyAsync(dd->p, d.data(), d.size() * sizeof(TtoDesc), hipMemcpyHostToDevice, X.s()),
        "descriptor upload");
  hipEvent_t e = X.t0();
  tto_apply_all(L, (const TtoDesc*)dd->p, blocks, X.s());
  X.t1(e, QTT_K_APPLY, flops, bytes);
  X.sync();  // the host descriptor array is released on return
  return z;
}

static TTP op_apply(const Ctx& X, const TT& A, const TT& x, int flags, const SketchOpts& o,
                    RoundStats* st);
static TTP identity_op(const Ctx& X, int bits, int d0 = 6);

// Rounding of an explicit train (e.g. a sum of two trains): with a rank cap
// the randomized sketch (identity operator) keeps every factorisation at the
// sketch size; without a cap (or in exact mode) the deterministic
// QR + SVD rounding is used.
static TTP round_any(const Ctx& X, const TTP& x, const SketchOpts& o, RoundStats* st) {
  if (o.cap > 0 && !o.exact && x->dout[0] <= 6) {
    auto I = identity_op(X, x->L - 1, x->dout[0]);
    return sketch_apply(X, *I, *x, o, st);
  }
  round_tt(X, *x, o.delta, o.cap, st);
  return x;
}

// Green step of Alg. 2 in bounded factors (see qtt_green_build):
// u = U x, s = Sd u, p = P s, q = u/(2 mu0) - (c/2) p, eps = E q.
static TTP amen_product(const Ctx& X, const TT& A, const TT& x, const SketchOpts& o, int slot, RoundStats* st);

static TTP green_chain(const Ctx& X, const TT& G, const TT& x, int flags, const SketchOpts& o,
                       RoundStats* st) {
  SketchOpts o2 = o;
  RoundStats s1;
  double disc = 0.0;
  // QTT_MV_AMEN: the four factor products by AMEn (rounded products of
  // Alg. 2's Green step, App. B), warm-started per factor
  const bool am = o.matvec == QTT_MV_AMEN && o.amen && !o.exact && o.cap > 0 && !(flags & (QTT_EXACT | QTT_NO_ROUND));
  auto prod = [&](const TT& A, const TT& v, int slot, RoundStats* sp) {
    return am ? amen_product(X, A, v, o2, slot, sp) : op_apply(X, A, v, flags, o2, sp);
  };
  o2.seed = o.seed * 7 + 1;
  auto u = prod(*G.gU, x, 0, &s1);
  disc = std::max(disc, s1.rel_max());
  o2.seed = o.seed * 7 + 2;
  auto s = prod(*G.gS, *u, 1, &s1);
  disc = std::max(disc, s1.rel_max());
  o2.seed = o.seed * 7 + 3;
  auto p = prod(*G.gP, *s, 2, &s1);
  disc = std::max(disc, s1.rel_max());
  TTP q;
  if (G.inv_mu0_b) {
    if (G.nbatch_scalars != x.B) throw std::invalid_argument("Green scalars do not match the batch");
    q = axpby(X, 1.0, *u, -1.0, *p, (const double*)G.inv_mu0_b->p, (const double*)G.c_b->p);
  } else {
    q = axpby(X, G.inv_mu0, *u, -G.c, *p);
  }
  if (!(flags & QTT_NO_ROUND)) {
    o2.seed = o.seed * 7 + 5;
    SketchOpts o3 = o2;
    if (flags & QTT_EXACT) o3.exact = true;
    q = round_any(X, q, o3, &s1);
    disc = std::max(disc, s1.rel_max());
  }
  o2.seed = o.seed * 7 + 4;
  o2.no_truncate = o.no_truncate;
  auto e = prod(*G.gE, *q, 3, st);
  if (st) {
    // fold the intermediate roundings into the reported maximum
    for (size_t b = 0; b < st->disc2.size(); ++b)
      st->disc2[b] = std::max(st->disc2[b], disc * disc * st->norm[b] * st->norm[b]);
  }
  return e;
}

static TTP op_apply(const Ctx& X, const TT& A, const TT& x, int flags, const SketchOpts& o,
                    RoundStats* st) {
  if (A.kind == 2) return green_chain(X, A, x, flags, o, st);
  if (A.kind != 1) throw std::invalid_argument("not an operator");
  if (flags & QTT_NO_ROUND) return apply_full(X, A, x);
  SketchOpts o2 = o;
  if (flags & QTT_EXACT) o2.exact = true;
  return sketch_apply(X, A, x, o2, st);
}

// ---------------------------------------------------------------------------
// AMEn-adapted product y ~ A x (App. B)
// ---------------------------------------------------------------------------
static std::vector<double> diff_norms(const Ctx& X, const TT& a, const TT& b, double prev_rel);
static std::vector<std::complex<double>> tt_dot_diag(const Ctx& X, const TT& x, const TT& y);

// QR sweep right to left: cores 1..L-1 become right-orthonormal (orthonormal
// rows of the r_k x (d r_{k+1}) unfolding), the R factors move left; the
// tensor is unchanged.
static void orth_rl(const Ctx& X, TT& y) {
  const int L = y.L, B = y.B;
  for (int k = L - 1; k >= 1; --k) {
    const int p = y.r[k], q = y.dout[k] * y.r[k + 1];
    const int kk = std::min(p, q);
    const long msz = (long)p * q;
    // M^H (q x p) = Q R, so M = R^H Q^H
    auto Qb = X.buf((size_t)B * q * kk);
    auto R = X.buf((size_t)B * kk * p);
    auto ws = X.buf(qr_ws(B, q, p));
    ck_qr(X, B, q, p, MatView{y.core[k], 1, (long)q, msz, 1}, MatOut{(cplx*)R->p, (long)p, 1, (long)kk * p},
          MatOut{(cplx*)Qb->p, (long)kk, 1, (long)q * kk}, (cplx*)ws->p, X.s());
    auto nk = X.buf((size_t)B * kk * q);
    ck_conj_transpose(X, B, q, kk, MatView{(cplx*)Qb->p, (long)kk, 1, (long)q * kk, 0},
                      MatOut{(cplx*)nk->p, (long)q, 1, (long)kk * q}, X.s());
    const int rows = y.r[k - 1] * y.dout[k - 1];
    auto nk1 = X.buf((size_t)B * rows * kk);
    G(X, rows, kk, p, OP_N, y.core[k - 1], p, OP_C, (cplx*)R->p, p, (cplx*)nk1->p, kk, B, (long)rows * p,
      (long)kk * p, (long)rows * kk);
    set_core(X, y, k, kk, y.r[k + 1], nk);
    set_core(X, y, k - 1, y.r[k - 1], kk, nk1);
  }
}

// Left singular vectors U (B, m, kk) and singular values (host, B x kk,
// descending) of B matrices Y (m x n, row-major), kk = min(m, n): QR of the
// tall orientation, one-sided Jacobi of its square factor.
static BufP left_singular(const Ctx& X, int B, int m, int n, const cplx* Y, std::vector<double>& S) {
  const int kk = std::min(m, n);
  if (kk > 320) throw std::length_error("AMEn local core beyond the Jacobi size");
  auto R = X.buf((size_t)B * kk * kk);
  auto Sd = X.bufd((size_t)B * kk);
  auto U = X.buf((size_t)B * m * kk);
  const long ysz = (long)m * n;
  if (m >= n) {
    auto Q = X.buf((size_t)B * m * kk);
    auto ws = X.buf(qr_ws(B, m, n));
    ck_qr(X, B, m, n, MatView{Y, (long)n, 1, ysz, 0}, MatOut{(cplx*)R->p, (long)kk, 1, (long)kk * kk},
          MatOut{(cplx*)Q->p, (long)kk, 1, (long)m * kk}, (cplx*)ws->p, X.s());
    auto UR = X.buf((size_t)B * kk * kk);
    jacobi_any(X, B, kk, MatView{(cplx*)R->p, (long)kk, 1, (long)kk * kk, 0},
               MatOut{(cplx*)UR->p, (long)kk, 1, (long)kk * kk}, (double*)Sd->p);
    G(X, m, kk, kk, OP_N, (cplx*)Q->p, kk, OP_N, (cplx*)UR->p, kk, (cplx*)U->p, kk, B, (long)m * kk,
      (long)kk * kk, (long)m * kk);
  } else {
    // Y^H (n x m) = Q R, Y = R^H Q^H: the left singular vectors of R^H
    auto ws = X.buf(qr_ws(B, n, m));
    ck_qr(X, B, n, m, MatView{Y, 1, (long)n, ysz, 1}, MatOut{(cplx*)R->p, (long)kk, 1, (long)kk * kk},
          MatOut{nullptr, 0, 0, 0}, (cplx*)ws->p, X.s());
    jacobi_any(X, B, kk, MatView{(cplx*)R->p, 1, (long)kk, (long)kk * kk, 1},
               MatOut{(cplx*)U->p, (long)kk, 1, (long)kk * kk}, (double*)Sd->p);
  }
  S.resize((size_t)B * kk);
  check(hipMemcpyAsync(S.data(), Sd->p, S.size() * sizeof(double), hipMemcpyDeviceToHost, X.s()), "S d2h");
  X.sync();
  return U;
}

// One left-to-right AMEn sweep.  y and z are right-orthonormal (cores
// 1..L-1) on entry.  At core k the local solution is the projection of
// A x onto y's frame (the Galerkin condition: left interface Ly, right
// interface Wy), truncated by SVD at delta / sqrt(L - 1) of its norm and
// the cap; the residual A x - y is projected onto z's frame (its new core)
// and, with y's left and z's right frame, enriches the kept singular
// vectors before the QR that gives y's core.  On return y holds the
// enriched cores (left-orthonormal but the last), z the residual train,
// and kept the truncated rank of every bond.
static void amen_sweep(const Ctx& X, const TT& A, const TT& x, TT& y, TT& z, double delta, int cap,
                       std::vector<int>& kept, RoundStats* st = nullptr) {
  const int L = x.L, B = x.B;
  // right interfaces Wy[k] (B, rho_k, r_k, ry_k) and Wz[k] (B, rho_k, r_k,
  // rz_k) of A x against conj(y), conj(z) over the cores k..L-1; SRc[k]
  // (B, rz_k, ry_k) the conjugate of sum conj(z) y over the same cores
  std::vector<BufP> Wy(L + 1), Wz(L + 1), SRc(L + 1);
  for (auto* v : {&Wy, &Wz, &SRc}) {
    (*v)[L] = X.buf(B);
    ck_fill(X, (cplx*)(*v)[L]->p, B, C1(), X.s());
  }
  for (int k = L - 1; k >= 1; --k) {
    const int rho = A.r[k], r = x.r[k], d = A.dout[k];
    const int ry = y.r[k], ry2 = y.r[k + 1], rz = z.r[k], rz2 = z.r[k + 1];
    auto Xy = right_contract(X, A, x, k, (const cplx*)Wy[k + 1]->p, ry2);
    Wy[k] = X.buf((size_t)B * rho * r * ry);
    right_project(X, B, rho, r, d, ry2, (const cplx*)Xy->p, OP_C, y.core[k], y.celems(k), ry, (cplx*)Wy[k]->p);
    auto Xz = right_contract(X, A, x, k, (const cplx*)Wz[k + 1]->p, rz2);
    Wz[k] = X.buf((size_t)B * rho * r * rz);
    right_project(X, B, rho, r, d, rz2, (const cplx*)Xz->p, OP_C, z.core[k], z.celems(k), rz, (cplx*)Wz[k]->p);
    // T = y_k SR[k+1]^T (ry d x rz2); SRc[k] = z_k T^H
    auto T = X.buf((size_t)B * ry * d * rz2);
    G(X, ry * d, rz2, ry2, OP_N, y.core[k], ry2, OP_C, (cplx*)SRc[k + 1]->p, ry2, (cplx*)T->p, rz2, B,
      y.celems(k), (long)rz2 * ry2, (long)ry * d * rz2);
    SRc[k] = X.buf((size_t)B * rz * ry);
    G(X, rz, ry, d * rz2, OP_N, z.core[k], (long)d * rz2, OP_C, (cplx*)T->p, (long)d * rz2, (cplx*)SRc[k]->p, ry,
      B, z.celems(k), (long)ry * d * rz2, (long)rz * ry);
  }
  BufP Ly = X.buf(B), Lz = X.buf(B), SL = X.buf(B);
  for (auto* v : {&Ly, &Lz, &SL}) ck_fill(X, (cplx*)(*v)->p, B, C1(), X.s());
  kept.assign(L + 1, 1);
  const double tscale = delta / std::sqrt((double)std::max(L - 1, 1));
  std::vector<double> disc2(B, 0.0), norm(B, 0.0);
  for (int k = 0; k < L; ++k) {
    const int d = A.dout[k], rho2 = A.r[k + 1], r2 = x.r[k + 1];
    const int ry = y.r[k], ry2 = y.r[k + 1], rz = z.r[k], rz2 = z.r[k + 1];
    const int m = ry * d, mz = rz * d;
    const long pr = (long)rho2 * r2;
    auto Py = left_step(X, A, x, k, (const cplx*)Ly->p, ry);  // (B, ry, d, rho2, r2)
    auto Pz = left_step(X, A, x, k, (const cplx*)Lz->p, rz);
    // Galerkin solution (B, m, ry2) and the residual in z's frame (B, mz, rz2)
    auto Yk = X.buf((size_t)B * m * ry2);
    G(X, m, ry2, (int)pr, OP_N, (cplx*)Py->p, pr, OP_N, (cplx*)Wy[k + 1]->p, ry2, (cplx*)Yk->p, ry2, B,
      (long)m * pr, pr * ry2, (long)m * ry2);
    auto Zk = X.buf((size_t)B * mz * rz2);
    G(X, mz, rz2, (int)pr, OP_N, (cplx*)Pz->p, pr, OP_N, (cplx*)Wz[k + 1]->p, rz2, (cplx*)Zk->p, rz2, B,
      (long)mz * pr, pr * rz2, (long)mz * rz2);
    if (k == L - 1) {
      // Zk -= SL Yk (the right interfaces are 1 here)
      G(X, rz, d, ry, OP_N, (cplx*)SL->p, ry, OP_N, (cplx*)Yk->p, d, (cplx*)Zk->p, d, B, (long)rz * ry,
        (long)m, (long)mz, 1, 0, 0, 0, CR(-1.0), C1());
      set_core(X, y, k, ry, 1, Yk);
      set_core(X, z, k, rz, 1, Zk);
      if (st) {
        st->disc2 = disc2;
        st->norm = norm;
      }
      break;
    }
    // truncation of the local solution (its norm is that of the singular
    // values: one host transfer per core)
    std::vector<double> S;
    auto U = left_singular(X, B, m, ry2, (const cplx*)Yk->p, S);
    const int kk = std::min(m, ry2);
    std::vector<double> nrm(B, 0.0);
    for (int b = 0; b < B; ++b) {
      for (int j = 0; j < kk; ++j) nrm[b] += S[(size_t)b * kk + j] * S[(size_t)b * kk + j];
      nrm[b] = std::sqrt(nrm[b]);
      if (!std::isfinite(nrm[b])) throw nan_error("NaN/Inf in an AMEn local core");
    }
    std::vector<double> thr(B);
    for (int b = 0; b < B; ++b) {
      thr[b] = tscale * nrm[b];
      norm[b] = nrm[b];
    }
    const int r = choose_rank(S, B, kk, thr, cap, disc2);
    kept[k + 1] = r;
    // Yt = U_r U_r^H Yk, the truncated local core
    auto Cc = X.buf((size_t)B * r * ry2);
    G(X, r, ry2, m, OP_C, (cplx*)U->p, kk, OP_N, (cplx*)Yk->p, ry2, (cplx*)Cc->p, ry2, B, (long)m * kk,
      (long)m * ry2, (long)r * ry2);
    auto Yt = X.buf((size_t)B * m * ry2);
    G(X, m, ry2, r, OP_N, (cplx*)U->p, kk, OP_N, (cplx*)Cc->p, ry2, (cplx*)Yt->p, ry2, B, (long)m * kk,
      (long)r * ry2, (long)m * ry2);
    // Zk -= (SL Yt) SR[k+1]^T
    auto T1 = X.buf((size_t)B * rz * d * ry2);
    G(X, rz, d * ry2, ry, OP_N, (cplx*)SL->p, ry, OP_N, (cplx*)Yt->p, (long)d * ry2, (cplx*)T1->p,
      (long)d * ry2, B, (long)rz * ry, (long)m * ry2, (long)rz * d * ry2);
    G(X, mz, rz2, ry2, OP_N, (cplx*)T1->p, ry2, OP_C, (cplx*)SRc[k + 1]->p, ry2, (cplx*)Zk->p, rz2, B,
      (long)mz * ry2, (long)rz2 * ry2, (long)mz * rz2, 1, 0, 0, 0, CR(-1.0), C1());
    // enrichment [U_r, Py Wz[k+1] - Yt SR[k+1]^T] (B, m, r + rz2)
    const int ke = r + rz2;
    auto UE = X.buf((size_t)B * m * ke);
    ck_copy2d(X, B, m, r, MatView{(cplx*)U->p, (long)kk, 1, (long)m * kk, 0},
              MatOut{(cplx*)UE->p, (long)ke, 1, (long)m * ke}, C1(), X.s());
    G(X, m, rz2, (int)pr, OP_N, (cplx*)Py->p, pr, OP_N, (cplx*)Wz[k + 1]->p, rz2, (cplx*)UE->p + r, ke, B,
      (long)m * pr, pr * rz2, (long)m * ke);
    G(X, m, rz2, ry2, OP_N, (cplx*)Yt->p, ry2, OP_C, (cplx*)SRc[k + 1]->p, ry2, (cplx*)UE->p + r, ke, B,
      (long)m * ry2, (long)rz2 * ry2, (long)m * ke, 1, 0, 0, 0, CR(-1.0), C1());
    const int kq = std::min(m, ke);
    auto Q = X.buf((size_t)B * m * kq);
    {
      auto R = X.buf((size_t)B * kq * ke);
      auto ws = X.buf(qr_ws(B, m, ke));
      ck_qr(X, B, m, ke, MatView{(cplx*)UE->p, (long)ke, 1, (long)m * ke, 0},
            MatOut{(cplx*)R->p, (long)ke, 1, (long)kq * ke}, MatOut{(cplx*)Q->p, (long)kq, 1, (long)m * kq},
            (cplx*)ws->p, X.s());
    }
    const int kz = std::min(mz, rz2);
    auto Qz = X.buf((size_t)B * mz * kz);
    {
      auto R = X.buf((size_t)B * kz * rz2);
      auto ws = X.buf(qr_ws(B, mz, rz2));
      ck_qr(X, B, mz, rz2, MatView{(cplx*)Zk->p, (long)rz2, 1, (long)mz * rz2, 0},
            MatOut{(cplx*)R->p, (long)rz2, 1, (long)kz * rz2}, MatOut{(cplx*)Qz->p, (long)kz, 1, (long)mz * kz},
            (cplx*)ws->p, X.s());
    }
    // left interfaces through core k
    auto Ly2 = X.buf((size_t)B * kq * pr);
    G(X, kq, (int)pr, m, OP_C, (cplx*)Q->p, kq, OP_N, (cplx*)Py->p, pr, (cplx*)Ly2->p, pr, B, (long)m * kq,
      (long)m * pr, (long)kq * pr);
    auto Lz2 = X.buf((size_t)B * kz * pr);
    G(X, kz, (int)pr, mz, OP_C, (cplx*)Qz->p, kz, OP_N, (cplx*)Pz->p, pr, (cplx*)Lz2->p, pr, B, (long)mz * kz,
      (long)mz * pr, (long)kz * pr);
    auto T2 = X.buf((size_t)B * rz * d * kq);
    G(X, rz, d * kq, ry, OP_N, (cplx*)SL->p, ry, OP_N, (cplx*)Q->p, (long)d * kq, (cplx*)T2->p, (long)d * kq, B,
      (long)rz * ry, (long)m * kq, (long)rz * d * kq);
    auto SL2 = X.buf((size_t)B * kz * kq);
    G(X, kz, kq, mz, OP_C, (cplx*)Qz->p, kz, OP_N, (cplx*)T2->p, kq, (cplx*)SL2->p, kq, B, (long)mz * kz,
      (long)mz * kq, (long)kz * kq);
    // core k of y and z; core k + 1 keeps its old left rank until its
    // own step replaces it
    set_core(X, y, k, ry, kq, Q);
    set_core(X, z, k, rz, kz, Qz);
    Ly = Ly2;
    Lz = Lz2;
    SL = SL2;
  }
}

// Deep copy of a train (cores into new buffers).
static TTP copy_tt(const Ctx& X, const TT& x) {
  auto t = new_tt(X, x.L, x.B, x.dout, x.r);
  for (int k = 0; k < x.L; ++k)
    check(hipMemcpyAsync(t->core[k], x.core[k], (size_t)x.B * x.celems(k) * sizeof(cplx), hipMemcpyDeviceToDevice,
                         X.s()),
          "train copy");
  return t;
}

// The product without its enrichment: on every bond the first kept[k]
// columns of the enriched basis (they span the kept singular vectors) and
// the matching rows of the next core.
static TTP amen_compact(const Ctx& X, const TT& y, const std::vector<int>& kept) {
  auto t = new_tt(X, y.L, y.B, y.dout, kept);
  for (int k = 0; k < y.L; ++k) {
    const int r0 = y.r[k], d = y.dout[k], r1 = y.r[k + 1];
    ck_copy2d(X, y.B, kept[k] * d, kept[k + 1], MatView{y.core[k], (long)r1, 1, (long)r0 * d * r1, 0},
              MatOut{t->core[k], (long)kept[k + 1], 1, (long)kept[k] * d * kept[k + 1]}, C1(), X.s());
  }
  return t;
}

struct AmenInfo {
  int sweeps = 0;
  double change = INFINITY;
};

// y ~ A x by AMEn sweeps from the initial guesses y0 and z0 (same batch and
// dimensions as the product), truncation delta and cap, at most `sweeps`
// sweeps, stopped when the product changes by less than tol (relative,
// largest over the batch) between two sweeps.
static TTP amen_apply(const Ctx& X, const TT& A, const TT& x, const TT& y0, const TT& z0, double delta, int cap,
                      int sweeps, double tol, AmenInfo* info, TTP* z_out = nullptr, RoundStats* st = nullptr) {
  const int L = x.L, B = x.B;
  if (A.kind != 1 || A.L != L) throw std::invalid_argument("AMEn: operator and train differ");
  if (B % A.opb) throw std::invalid_argument("train batch not a multiple of the operator instances");
  for (const TT* t : {&y0, &z0}) {
    if (t->kind != 0 || t->L != L || t->B != B) throw std::invalid_argument("AMEn: initial guess shape");
    for (int k = 0; k < L; ++k)
      if (t->dout[k] != A.dout[k]) throw std::invalid_argument("AMEn: initial guess dims");
  }
  for (int k = 0; k < L; ++k)
    if (A.din[k] != x.dout[k]) throw std::invalid_argument("operator input dim mismatch");
  auto y = copy_tt(X, y0), z = copy_tt(X, z0);
  orth_rl(X, *y);
  orth_rl(X, *z);
  TTP out, prev;
  AmenInfo inf;
  for (int m = 1; m <= std::max(1, sweeps); ++m) {
    std::vector<int> kept;
    amen_sweep(X, A, x, *y, *z, delta, cap, kept, st);
    out = amen_compact(X, *y, kept);
    inf.sweeps = m;
    if (prev) {
      // while the change is large, inner products (no QR sweep) measure it;
      // near the tolerance the difference train's norm does (no
      // cancellation)
      const bool gram = std::isfinite(inf.change) ? inf.change > 1e-4 : true;
      auto dn = diff_norms(X, *out, *prev, gram ? 1.0 : 0.0);
      std::vector<double> nn(B);
      if (gram) {
        auto d = tt_dot_diag(X, *out, *out);
        for (int b = 0; b < B; ++b) nn[b] = std::sqrt(std::max(0.0, d[b].real()));
      } else {
        nn = tt_norms(X, *out);
      }
      double ch = 0.0;
      for (int b = 0; b < B; ++b) ch = std::max(ch, dn[b] / std::max(nn[b], 1e-300));
      inf.change = ch;
      if (ch < tol && !(gram && ch < 1e-4)) break;
      if (gram && ch < tol) {
        // confirm a small change without cancellation
        auto de = diff_norms(X, *out, *prev, 0.0);
        auto ne = tt_norms(X, *out);
        ch = 0.0;
        for (int b = 0; b < B; ++b) ch = std::max(ch, de[b] / std::max(ne[b], 1e-300));
        inf.change = ch;
        if (ch < tol) break;
      }
    }
    prev = out;
    if (m < sweeps) {
      // fresh trains (the sweep's set_core calls keep every replaced core)
      y = copy_tt(X, *y);
      z = copy_tt(X, *z);
      orth_rl(X, *y);
      orth_rl(X, *z);
    }
  }
  if (info) *info = inf;
  if (z_out) *z_out = z;
  return out;
}

// Warm starts of the AMEn products of a fixed-point loop: the last result
// and residual train of every product slot.
struct AmenSlots {
  std::map<int, std::pair<TTP, TTP>> yz;
  int sweeps = 6;       // cold start: at most this many sweeps
  int warm_sweeps = 3;  // warm start: at most this many sweeps
  int kick = 16;        // rank of the residual train (16: its products reach the matrix cores)
  // the sweeps stop when the product changes by less than this (relative)
  // between two sweeps; the loop ties it to its last relative update
  double tol = 1e-3;
};

// Random complex Gaussian train (cores scaled by 1 / sqrt(d r_{k+1})) with
// the given ranks, from the sketch generator's stream.
static TTP random_train(const Ctx& X, int L, int B, const std::vector<int>& dims, const std::vector<int>& ranks,
                        uint64_t seed) {
  auto t = new_tt(X, L, B, dims, ranks);
  GaussBlocks gb;
  gb.start[0] = 0;
  for (int k = 0; k < L; ++k) {
    const long cnt = (long)B * t->celems(k);
    gb.out[gb.n] = t->core[k];
    gb.stream[gb.n] = (uint64_t)k;
    gb.scale[gb.n] = 1.0 / std::sqrt((double)dims[k] * ranks[k + 1]);
    gb.start[gb.n + 1] = gb.start[gb.n] + cnt;
    if (++gb.n == GAUSS_MULTI_MAX) {
      gaussian_multi(gb, seed, X.s());
      gb.n = 0;
    }
  }
  gaussian_multi(gb, seed, X.s());
  return t;
}

static std::vector<int> capped_ranks(const std::vector<int>& dims, int r) {
  const int L = (int)dims.size();
  std::vector<int> rk(L + 1, 1);
  long left = 1;
  for (int k = 1; k < L; ++k) {
    left = std::min<long>(left * dims[k - 1], 1L << 30);
    long right = 1;
    for (int j = k; j < L && right < (1L << 30); ++j) right *= dims[j];
    rk[k] = (int)std::max<long>(1, std::min<long>(r, std::min(left, right)));
  }
  return rk;
}

// One product of the Green step by AMEn: the previous result in this slot
// (same batch) is the initial guess, else a random train at the cap's
// ranks; sweeps run until the product settles to the loop's tolerance.
// The residual train is carried the same way.
static TTP amen_product(const Ctx& X, const TT& A, const TT& x, const SketchOpts& o, int slot, RoundStats* st) {
  AmenSlots& am = *o.amen;
  auto& prev = am.yz[slot];
  const int L = x.L, B = x.B;
  const bool warm = prev.first && prev.second && prev.first->B == B && prev.first->dout == A.dout;
  TTP y0 = warm ? prev.first : random_train(X, L, B, A.dout, capped_ranks(A.dout, o.cap), o.seed * 31 + 7);
  TTP z0 = warm ? prev.second : random_train(X, L, B, A.dout, capped_ranks(A.dout, am.kick), o.seed * 31 + 11);
  AmenInfo inf;
  TTP z;
  auto y = amen_apply(X, A, x, *y0, *z0, o.delta, o.cap, warm ? am.warm_sweeps : am.sweeps,
                      std::max(o.delta, am.tol), &inf, &z, st);
  prev = std::make_pair(y, z);
  return y;
}

// Volume average of A(x) : x -> host (B x 6) complex; A's core 0 is 6x6.
static std::vector<std::complex<double>> mean_apply(const Ctx& X, const TT& A, const TT& x) {
  const int L = x.L, B = x.B;
  const int V = A.dout[0];
  if ((V != 6 && V != 3) || A.kind != 1) throw std::invalid_argument("mean_apply: needs a Voigt operator");
  auto one = X.buf(B);
  ck_fill(X, (cplx*)one->p, B, C1(), X.s());
  // core 0: P (B, 1, V, rho1, r1) -> Mc (B, V, rho1, r1)
  BufP Mc = left_step(X, A, x, 0, (cplx*)one->p, 1);
  const int lt = V;
  for (int k = 1; k < L; ++k) {
    // treat the Voigt output index as the sketch index (lt = 6)
    const int rho2 = A.r[k + 1], r2 = x.r[k + 1], d = A.dout[k];
    auto P = left_step(X, A, x, k, (cplx*)Mc->p, lt);
    auto Mn = X.buf((size_t)B * lt * rho2 * r2);
    ck_sum_middle(X, B, lt, d, rho2 * r2, (cplx*)P->p, (cplx*)Mn->p, CR(1.0 / d), X.s());
    Mc = Mn;
  }
  std::vector<std::complex<double>> out((size_t)B * V);
  check(hipMemcpyAsync(out.data(), Mc->p, out.size() * sizeof(cplx), hipMemcpyDeviceToHost, X.s()), "mean d2h");
  X.sync();
  return out;
}

// Gram matrix of inner products <x_a, y_b> = sum conj(x_a) y_b -> host (Bx x By)
static std::vector<std::complex<double>> tt_gram(const Ctx& X, const TT& x, const TT& y) {
  const int L = x.L, Bx = x.B, By = y.B;
  auto Mc = X.buf((size_t)Bx * By);
  ck_fill(X, (cplx*)Mc->p, (size_t)Bx * By, C1(), X.s());
  for (int k = 0; k < L; ++k) {
    const int rx = x.r[k], rx2 = x.r[k + 1], ry = y.r[k], ry2 = y.r[k + 1], d = x.dout[k];
    auto T = X.buf((size_t)Bx * By * rx * d * ry2);
    G(X, rx, d * ry2, ry, OP_N, (cplx*)Mc->p, ry, OP_N, y.core[k], (long)d * ry2, (cplx*)T->p,
      (long)d * ry2, Bx, (long)By * rx * ry, 0, (long)By * rx * d * ry2, By, (long)rx * ry,
      (long)ry * d * ry2, (long)rx * d * ry2);
    auto Mn = X.buf((size_t)Bx * By * rx2 * ry2);
    G(X, rx2, ry2, rx * d, OP_C, x.core[k], rx2, OP_N, (cplx*)T->p, ry2, (cplx*)Mn->p, ry2, Bx,
      (long)rx * d * rx2, (long)By * rx * d * ry2, (long)By * rx2 * ry2, By, 0,
      (long)rx * d * ry2, (long)rx2 * ry2);
    Mc = Mn;
  }
  std::vector<std::complex<double>> out((size_t)Bx * By);
  check(hipMemcpyAsync(out.data(), Mc->p, out.size() * sizeof(cplx), hipMemcpyDeviceToHost, X.s()), "gram d2h");
  X.sync();
  return out;
}

// Per-batch-element inner products <x_b, y_b> = sum conj(x_b) y_b (trains of
// the same batch): left-to-right contraction, two GEMMs per core.
static std::vector<std::complex<double>> tt_dot_diag(const Ctx& X, const TT& x, const TT& y) {
  const int L = x.L, B = x.B;
  if (y.L != L || y.B != B) throw std::invalid_argument("tt_dot_diag: shape mismatch");
  auto Mc = X.buf(B);
  ck_fill(X, (cplx*)Mc->p, B, C1(), X.s());
  for (int k = 0; k < L; ++k) {
    const int rx = x.r[k], rx2 = x.r[k + 1], ry = y.r[k], ry2 = y.r[k + 1], d = x.dout[k];
    // T (B, rx, d, ry2) = Mc (B, rx, ry) * y_k (B, ry, d ry2)
    auto T = X.buf((size_t)B * rx * d * ry2);
    G(X, rx, d * ry2, ry, OP_N, (cplx*)Mc->p, ry, OP_N, y.core[k], (long)d * ry2, (cplx*)T->p,
      (long)d * ry2, B, (long)rx * ry, (long)ry * d * ry2, (long)rx * d * ry2);
    // Mn (B, rx2, ry2) = x_k^H (rx2, rx d) * T (rx d, ry2)
    auto Mn = X.buf((size_t)B * rx2 * ry2);
    G(X, rx2, ry2, rx * d, OP_C, x.core[k], rx2, OP_N, (cplx*)T->p, ry2, (cplx*)Mn->p, ry2, B,
      (long)rx * d * rx2, (long)rx * d * ry2, (long)rx2 * ry2);
    Mc = Mn;
  }
  std::vector<std::complex<double>> out(B);
  check(hipMemcpyAsync(out.data(), Mc->p, B * sizeof(cplx), hipMemcpyDeviceToHost, X.s()), "dot d2h");
  X.sync();
  return out;
}

// ||a_b - b_b|| per batch element.  While the previous relative update is
// large the norms come from inner products (two GEMMs per core, no QR): the
// cancellation in <a,a> + <b,b> - 2 Re <a,b> costs a relative error of
// about eps * ||a||^2 / ||a - b||^2, below 1e-8 for updates above 1e-4.
// Small updates use the QR sweep of the difference train.
static std::vector<double> diff_norms(const Ctx& X, const TT& a, const TT& b, double prev_rel) {
  if (prev_rel > 1e-4) {
    auto aa = tt_dot_diag(X, a, a), bb = tt_dot_diag(X, b, b), ab = tt_dot_diag(X, a, b);
    std::vector<double> out(a.B);
    for (int i = 0; i < a.B; ++i)
      out[i] = std::sqrt(std::max(0.0, aa[i].real() + bb[i].real() - 2.0 * ab[i].real()));
    return out;
  }
  auto d = axpby(X, 1.0, a, -1.0, b);
  return tt_norms(X, *d);
}

// ---------------------------------------------------------------------------
// operator upload
// ---------------------------------------------------------------------------
static TTP upload_op(const Ctx& X, const host::HTT& h) {
  auto t = std::make_shared<TT>();
  const int L = (int)h.size();
  t->kind = 1; t->L = L; t->B = 1; t->pool = X.c->pool;
  t->dout.resize(L); t->din.resize(L); t->diag.resize(L); t->r.resize(L + 1);
  t->core.resize(L); t->coreR.assign(L, nullptr);
  for (int k = 0; k < L; ++k) {
    const host::HCore& c = h[k];
    t->r[k] = c.r0; t->r[k + 1] = c.r1; t->dout[k] = c.dout;
    t->diag[k] = (c.din == 0);
    t->din[k] = c.din == 0 ? c.dout : c.din;
    if (t->diag[k]) {
      auto b = X.buf(c.v.size());
      check(hipMemcpyAsync(b->p, c.v.data(), c.v.size() * sizeof(cplx), hipMemcpyHostToDevice, X.s()), "op h2d");
      t->core[k] = (cplx*)b->p;
      t->mem.push_back(b);
    } else {
      // host layout (r0, dout, din, r1) == layout R; build layout L (r0, din, dout, r1)
      std::vector<std::complex<double>> Lv(c.v.size());
      for (int a = 0; a < c.r0; ++a)
        for (int o = 0; o < c.dout; ++o)
          for (int i = 0; i < c.din; ++i)
            for (int b2 = 0; b2 < c.r1; ++b2)
              Lv[(((size_t)a * c.din + i) * c.dout + o) * c.r1 + b2] =
                  c.v[(((size_t)a * c.dout + o) * c.din + i) * c.r1 + b2];
      auto bl = X.buf(c.v.size());
      auto br = X.buf(c.v.size());
      check(hipMemcpyAsync(bl->p, Lv.data(), Lv.size() * sizeof(cplx), hipMemcpyHostToDevice, X.s()), "op h2d");
      check(hipMemcpyAsync(br->p, c.v.data(), c.v.size() * sizeof(cplx), hipMemcpyHostToDevice, X.s()), "op h2d");
      t->core[k] = (cplx*)bl->p;
      t->coreR[k] = (cplx*)br->p;
      t->mem.push_back(bl);
      t->mem.push_back(br);
    }
  }
  X.sync();
  return t;
}

static host::HTT adjoint_host(const host::HTT& h) {
  host::HTT out = h;
  for (auto& c : out) {
    if (c.din == 0) {
      for (auto& v : c.v) v = std::conj(v);
      continue;
    }
    for (int a = 0; a < c.r0; ++a)
      for (int o = 0; o < c.dout; ++o)
        for (int i = 0; i < c.din; ++i)
          for (int b = 0; b < c.r1; ++b)
            c.v[(((size_t)a * c.din + i) * c.dout + o) * c.r1 + b] =
                std::conj(h[&c - &out[0]].v[(((size_t)a * c.dout + o) * c.din + i) * c.r1 + b]);
    std::swap(c.dout, c.din);
  }
  return out;
}

// SFFT on `dim` axes (3, or 2 for plane problems) with the Voigt identity
// (6 or 3 components) on the control core
static TTP sfft_op(const Ctx& X, int n, double delta, int dim = 3) {
  host::HTT q = host::qn_tto(n, delta);
  host::HTT S;
  host::HCore id;
  const int V = dim == 2 ? 3 : 6;
  id.r0 = 1; id.dout = V; id.din = V; id.r1 = 1;
  id.v.assign((size_t)V * V, 0.0);
  for (int i = 0; i < V; ++i) id.v[i * V + i] = 1.0;
  S.push_back(id);
  for (int a = 0; a < dim; ++a)
    for (auto& c : q) S.push_back(c);
  auto t = upload_op(X, S);
  t->adj = upload_op(X, adjoint_host(S));
  return t;
}

static bool device_direction(const Ctx& X, int n, double delta, host::HTT& out);
static bool device_direction_staggered(const Ctx& X, int n, double delta, host::HTT& out);

// The Green factors from the direction train: its TT-SVD on the device, or
// (direct scheme) on the host when a bond rank exceeds the device path
static bool device_direction2d(const Ctx& X, int n, double delta, host::HTT& out);
static bool device_direction_staggered2d(const Ctx& X, int n, double delta, host::HTT& out);

static TTP green_op(const Ctx& X, int n, double lam0, double mu0, double delta, int scheme, int dim = 3) {
  host::HTT nt;
  host::GreenFactors gf;
  if (dim == 2 && scheme == QTT_SCHEME_STAGGERED) {
    if (!device_direction_staggered2d(X, n, delta, nt))
      throw std::length_error("plane staggered Green operator: direction-train rank beyond the device TT-SVD");
    gf = host::green_factors_staggered2d_from(nt, lam0, mu0);
  } else if (dim == 2) {
    if (!device_direction2d(X, n, delta, nt)) {
      // host TT-SVD of the 4 x 2^(2n) direction field (bonds beyond the
      // device path)
      const int N = 1 << n;
      const size_t NN = (size_t)N * N;
      std::vector<double> f, f2;
      host::momentum_freqs(n, f, f2);
      std::vector<double> T(4 * NN);
      for (int x = 0; x < N; ++x)
        for (int y = 0; y < N; ++y) {
          const size_t e = (size_t)x * N + y;
          const double r2 = f[x] * f[x] + f[y] * f[y];
          const double inv = r2 > 0 ? 1.0 / std::sqrt(r2) : 0.0;
          T[0 * NN + e] = f[x] * inv;
          T[1 * NN + e] = f[y] * inv;
          T[2 * NN + e] = f2[x] * inv;
          T[3 * NN + e] = f2[y] * inv;
        }
      std::vector<int> dims(2 * n + 1, 2);
      dims[0] = 4;
      nt = host::tt_svd_real(T, dims, delta, 0);
    }
    gf = host::green_factors2d_from(nt, lam0, mu0);
  } else if (scheme == QTT_SCHEME_STAGGERED) {
    if (!device_direction_staggered(X, n, delta, nt))
      throw std::length_error("staggered Green operator: direction-train rank beyond the device TT-SVD");
    gf = host::green_factors_staggered_from(nt, lam0, mu0);
  } else {
    gf = device_direction(X, n, delta, nt) ? host::green_factors_from(nt, lam0, mu0)
                                           : host::green_factors(n, lam0, mu0, delta);
  }
  auto t = std::make_shared<TT>();
  t->scheme = scheme;
  t->kind = 2; t->L = dim * n + 1; t->B = 1; t->pool = X.c->pool;
  t->gU = upload_op(X, gf.U);
  t->gS = upload_op(X, gf.Sd);
  t->gP = upload_op(X, gf.P);
  t->gE = upload_op(X, gf.E);
  t->inv_mu0 = gf.inv_2mu0;
  t->c = gf.half_c;
  t->dout = t->gE->dout; t->din = t->gU->din; t->diag = t->gU->diag;
  t->r = t->gU->r;
  return t;
}

// SFFT of a grid size, built once per (n, dim, delta) in a context
static TTP sfft_cached(const Ctx& X, int n, double delta, int dim = 3) {
  const auto key = std::make_pair(4 * n + dim, delta);
  auto it = X.c->sfft_cache.find(key);
  if (it != X.c->sfft_cache.end()) return it->second;
  auto t = sfft_op(X, n, delta, dim);
  X.c->sfft_cache[key] = t;
  return t;
}

// Green operator for one reference medium: the factors are built once per
// (n, delta, scheme) and shared, the two medium scalars are set per call
static TTP green_cached(const Ctx& X, int n, double lam0, double mu0, double delta, int scheme, int dim = 3) {
  const auto key = std::make_tuple(4 * n + dim, delta, scheme);
  auto it = X.c->green_cache.find(key);
  TTP base;
  if (it != X.c->green_cache.end()) {
    base = it->second;
  } else {
    base = green_op(X, n, lam0, mu0, delta, scheme, dim);
    X.c->green_cache[key] = base;
  }
  auto t = std::make_shared<TT>(*base);
  host::green_scalars_scheme(scheme, lam0, mu0, &t->inv_mu0, &t->c);
  return t;
}

// Green operator for a batch of structures (train batch = 6 per structure)
static TTP green_batch(const Ctx& X, int n, double delta, const std::vector<double>& lam0,
                       const std::vector<double>& mu0, int per, int scheme, int dim = 3) {
  auto t = green_cached(X, n, lam0[0], mu0[0], delta, scheme, dim);
  const int S = (int)lam0.size(), B = S * per;
  std::vector<double> a(B), c(B);
  for (int s2 = 0; s2 < S; ++s2) {
    double inv, hc;
    host::green_scalars_scheme(scheme, lam0[s2], mu0[s2], &inv, &hc);
    for (int q = 0; q < per; ++q) {
      a[(size_t)s2 * per + q] = inv;
      c[(size_t)s2 * per + q] = hc;
    }
  }
  t->inv_mu0_b = X.bufd(B);
  t->c_b = X.bufd(B);
  check(hipMemcpyAsync(t->inv_mu0_b->p, a.data(), B * sizeof(double), hipMemcpyHostToDevice, X.s()), "h2d");
  check(hipMemcpyAsync(t->c_b->p, c.data(), B * sizeof(double), hipMemcpyHostToDevice, X.s()), "h2d");
  X.sync();
  t->nbatch_scalars = B;
  return t;
}

// Several host operators of one structure pattern stacked as instances of
// one device operator, each zero-padded to the common ranks (exact).
static TTP upload_op_batch(const Ctx& X, const std::vector<host::HTT>& hs) {
  const int S = (int)hs.size();
  if (S == 1) return upload_op(X, hs[0]);
  const int L = (int)hs[0].size();
  auto t = std::make_shared<TT>();
  t->kind = 1; t->L = L; t->B = 1; t->opb = S; t->pool = X.c->pool;
  t->dout.resize(L); t->din.resize(L); t->diag.resize(L); t->r.assign(L + 1, 1);
  t->core.resize(L); t->coreR.assign(L, nullptr);
  for (int k = 0; k < L; ++k) {
    const host::HCore& c0 = hs[0][k];
    t->dout[k] = c0.dout;
    t->diag[k] = (c0.din == 0);
    t->din[k] = c0.din == 0 ? c0.dout : c0.din;
    for (int s2 = 0; s2 < S; ++s2) {
      const host::HCore& c = hs[s2][k];
      if ((int)hs[s2].size() != L || c.dout != c0.dout || c.din != c0.din)
        throw std::invalid_argument("batched operators differ in structure");
      t->r[k] = std::max(t->r[k], c.r0);
      t->r[k + 1] = std::max(t->r[k + 1], c.r1);
    }
  }
  for (int k = 0; k < L; ++k) {
    const int R0 = t->r[k], R1 = t->r[k + 1], d = t->dout[k];
    const int e = t->diag[k] ? 1 : t->din[k];
    const size_t inst = (size_t)R0 * d * e * R1;
    std::vector<std::complex<double>> Lv(inst * S, 0.0), Rv;
    if (!t->diag[k]) Rv.assign(inst * S, 0.0);
    for (int s2 = 0; s2 < S; ++s2) {
      const host::HCore& c = hs[s2][k];
      std::complex<double>* lo = Lv.data() + inst * s2;
      for (int a = 0; a < c.r0; ++a)
        for (int o = 0; o < d; ++o)
          for (int i = 0; i < e; ++i)
            for (int b2 = 0; b2 < c.r1; ++b2) {
              if (t->diag[k]) {
                lo[((size_t)a * d + o) * R1 + b2] = c.v[((size_t)a * d + o) * c.r1 + b2];
              } else {
                const std::complex<double> v = c.v[(((size_t)a * d + o) * e + i) * c.r1 + b2];
                lo[(((size_t)a * e + i) * d + o) * R1 + b2] = v;                 // layout L
                Rv[inst * s2 + (((size_t)a * d + o) * e + i) * R1 + b2] = v;     // layout R
              }
            }
    }
    auto bl = X.buf(Lv.size());
    check(hipMemcpyAsync(bl->p, Lv.data(), Lv.size() * sizeof(cplx), hipMemcpyHostToDevice, X.s()), "op h2d");
    t->core[k] = (cplx*)bl->p;
    t->mem.push_back(bl);
    if (!t->diag[k]) {
      auto br = X.buf(Rv.size());
      check(hipMemcpyAsync(br->p, Rv.data(), Rv.size() * sizeof(cplx), hipMemcpyHostToDevice, X.s()), "op h2d");
      t->coreR[k] = (cplx*)br->p;
      t->mem.push_back(br);
    }
  }
  X.sync();
  return t;
}

// identity operator on a train of `bits` binary cores after a control core
// of d0 values
static TTP identity_op(const Ctx& X, int bits, int d0) {
  const auto key = std::make_pair(bits, d0);
  auto it = X.c->ident.find(key);
  if (it != X.c->ident.end()) return it->second;
  host::HTT h;
  host::HCore id;
  id.r0 = 1; id.dout = d0; id.din = d0; id.r1 = 1;
  id.v.assign((size_t)d0 * d0, 0.0);
  for (int i = 0; i < d0; ++i) id.v[i * d0 + i] = 1.0;
  h.push_back(id);
  for (int k = 0; k < bits; ++k) {
    host::HCore c;
    c.r0 = 1; c.dout = 2; c.din = 0; c.r1 = 1;
    c.v.assign(2, 1.0);
    h.push_back(c);
  }
  auto t = upload_op(X, h);
  X.c->ident[key] = t;
  return t;
}

// constant strain train: control core E (B x V), then `bits` cores of ones
static TTP const_strain(const Ctx& X, int n, int B, const double* E, int V = 6, int dim = 3) {
  const int L = dim * n + 1;
  std::vector<int> dims(L, 2), rk(L + 1, 1);
  dims[0] = V;
  auto t = new_tt(X, L, B, dims, rk);
  std::vector<std::complex<double>> e((size_t)B * V);
  for (int i = 0; i < B * V; ++i) e[i] = E[i];
  check(hipMemcpyAsync(t->core[0], e.data(), e.size() * sizeof(cplx), hipMemcpyHostToDevice, X.s()), "E h2d");
  for (int k = 1; k < L; ++k) ck_fill(X, t->core[k], (size_t)B * 2, C1(), X.s());
  X.sync();
  return t;
}

// d(C)/d(theta) as raised operator from the one-hot train: Voigt core
// D[I][J] * chi_0[p][alpha], spatial cores of chi.
static TTP dC_op(const Ctx& X, const host::HTT& chi, int p, const double* D, int V) {
  host::HTT h;
  host::HCore c0;
  const int r1 = chi[0].r1;
  c0.r0 = 1; c0.dout = V; c0.din = V; c0.r1 = r1;
  c0.v.assign((size_t)V * V * r1, 0.0);
  for (int I = 0; I < V * V; ++I)
    for (int a = 0; a < r1; ++a) c0.v[(size_t)I * r1 + a] = D[I] * chi[0].v[(size_t)p * r1 + a];
  h.push_back(c0);
  for (size_t k = 1; k < chi.size(); ++k) h.push_back(chi[k]);
  return upload_op(X, h);
}

static bool verbose() {
  // thread-safe static initialisation (load-case groups log from several
  // host threads)
  static const bool v = []() {
    const char* e = std::getenv("QTTHOM_VERBOSE");
    return e && *e && *e != '0';
  }();
  return v;
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// Lippmann-Schwinger solver (Alg. 2)
// ---------------------------------------------------------------------------
struct Ops {
  TTP S, G, Cd, I;
  host::HTT chi;
  double lam0 = 0, mu0 = 0;
};

// ---------------------------------------------------------------------------
// One-hot phase train on the device (the binary discretisation of Sec. 4.3
// followed by TT-SVD, recomputed per geometry as App. D notes)
// ---------------------------------------------------------------------------
// R (c x c) of the QR of a tall m x c matrix (row-major, contiguous) by a
// tree of batched QRs: blocks of b rows are factored, their R factors
// stacked and factored again until one block remains.  Orthogonal
// transformations throughout, so the singular values of R are those of the
// matrix to working accuracy.
static BufP tsqr_r(const Ctx& X, BufP M, long m, int c) {
  const int b = c <= 96 ? 256 : 2 * ((c + 15) / 16) * 16;  // rows per block (m >= c per block)
  while (m > b) {
    const long nb = (m + b - 1) / b;
    BufP src = M;
    if (nb * b != m) {
      // zero-pad the last block
      src = X.buf((size_t)nb * b * c);
      ck_fill(X, (cplx*)src->p + (size_t)m * c, (size_t)(nb * b - m) * c, C0(), X.s());
      ck_copy2d(X, 1, (int)m, c, MatView{(cplx*)M->p, c, 1, (long)m * c, 0},
                MatOut{(cplx*)src->p, c, 1, (long)nb * b * c}, C1(), X.s());
    }
    auto Rs = X.buf((size_t)nb * c * c);
    // workspace bounded to ~256 MB per launch
    const size_t per = qr_ws_per_matrix(b, c);
    const long chunk = std::max<long>(1, std::min<long>(nb, (long)((256UL << 20) / (16 * per))));
    auto ws = X.buf(qr_ws(chunk, b, c));
    for (long b0 = 0; b0 < nb; b0 += chunk) {
      const int cnt = (int)std::min(chunk, nb - b0);
      ck_qr(X, cnt, b, c, MatView{(cplx*)src->p + (size_t)b0 * b * c, c, 1, (long)b * c, 0},
            MatOut{(cplx*)Rs->p + (size_t)b0 * c * c, c, 1, (long)c * c}, MatOut{nullptr, 0, 0, 0},
            (cplx*)ws->p, X.s());
    }
    M = Rs;
    m = nb * c;
  }
  const int k = (int)std::min<long>(m, c);
  auto R = X.buf((size_t)c * c);
  ck_fill(X, (cplx*)R->p, (size_t)c * c, C0(), X.s());
  auto ws = X.buf(qr_ws(1, (int)m, c));
  ck_qr(X, 1, (int)m, c, MatView{(cplx*)M->p, c, 1, m * c, 0}, MatOut{(cplx*)R->p, c, 1, (long)c * c},
        MatOut{nullptr, 0, 0, 0}, (cplx*)ws->p, X.s());
  (void)k;
  return R;
}

// TT-SVD of the one-hot tensor chi[p, x] = (phase(x) == p) (Sec. 4.3
// binary discretisation) on the device; ||chi|| = sqrt(2^(3n)).
static bool device_ttsvd(const Ctx& X, BufP T, int bits, int P, double thr, host::HTT& out);

// one-hot phase train of a voxel (or pixel) array of 2^bits entries
static bool device_chi(const Ctx& X, const uint8_t* phase, bool on_device, int bits, int P, double delta,
                       host::HTT& out) {
  const long NN = 1L << bits;
  const int L = bits + 1;
  const uint8_t* dph = phase;
  BufP phb;
  if (!on_device) {
    phb = X.buf((size_t)(NN + 15) / 16);
    check(hipMemcpyAsync(phb->p, phase, NN, hipMemcpyHostToDevice, X.s()), "phase h2d");
    dph = (const uint8_t*)phb->p;
  }
  auto T = X.buf((size_t)P * NN);
  auto flag = X.bufd(1);
  check(hipMemsetAsync(flag->p, 0, sizeof(int), X.s()), "flag clear");
  need(X, T->p, (long)P * NN - 1, "onehot out");
  onehot(dph, NN, P, (cplx*)T->p, (int*)flag->p, X.s());
  int bad = 0;
  check(hipMemcpyAsync(&bad, flag->p, sizeof(int), hipMemcpyDeviceToHost, X.s()), "flag d2h");
  X.sync();
  if (bad) throw std::invalid_argument("phase id out of range");
  return device_ttsvd(X, T, bits, P, delta / std::sqrt((double)(L - 1)) * std::sqrt((double)NN), out);
}

// TT-SVD of the unit momentum directions n^sigma_a (App. A, the Green
// factors' shared train) on the device: every nonzero frequency contributes
// |n^0|^2 + |n^1|^2 = 2, so ||T|| = sqrt(2 (2^(3n) - 1)).
static bool device_direction(const Ctx& X, int n, double delta, host::HTT& out) {
  const long NN = 1L << (3 * n);
  const int L = 3 * n + 1, N = 1 << n;
  std::vector<double> f, f2;
  host::momentum_freqs(n, f, f2);
  auto fd = X.bufd(2 * (size_t)N);
  check(hipMemcpyAsync(fd->p, f.data(), N * sizeof(double), hipMemcpyHostToDevice, X.s()), "freq h2d");
  check(hipMemcpyAsync((double*)fd->p + N, f2.data(), N * sizeof(double), hipMemcpyHostToDevice, X.s()),
        "freq h2d");
  auto T = X.buf((size_t)6 * NN);
  need(X, T->p, 6 * NN - 1, "direction out");
  direction((const double*)fd->p, (const double*)fd->p + N, n, (cplx*)T->p, X.s());
  X.sync();  // the host frequency arrays are released on return
  return device_ttsvd(X, T, 3 * n, 6, delta / std::sqrt((double)(L - 1)) * std::sqrt(2.0 * (double)(NN - 1)),
                      out);
}

// The plane version: 4 x 2^(2n) directions (sigma, a), a in {x, y}
static bool device_direction2d(const Ctx& X, int n, double delta, host::HTT& out) {
  const long NN = 1L << (2 * n);
  const int L = 2 * n + 1, N = 1 << n;
  std::vector<double> f, f2;
  host::momentum_freqs(n, f, f2);
  auto fd = X.bufd(2 * (size_t)N);
  check(hipMemcpyAsync(fd->p, f.data(), N * sizeof(double), hipMemcpyHostToDevice, X.s()), "freq h2d");
  check(hipMemcpyAsync((double*)fd->p + N, f2.data(), N * sizeof(double), hipMemcpyHostToDevice, X.s()),
        "freq h2d");
  auto T = X.buf((size_t)4 * NN);
  need(X, T->p, 4 * NN - 1, "direction out");
  direction2d((const double*)fd->p, (const double*)fd->p + N, n, (cplx*)T->p, X.s());
  X.sync();
  return device_ttsvd(X, T, 2 * n, 4, delta / std::sqrt((double)(L - 1)) * std::sqrt(2.0 * (double)(NN - 1)),
                      out);
}

// The train of the staggered-grid directions (n_a, m_a) (App. A, Table 3):
// the field on the device from one axis's difference symbols, then the
// device TT-SVD (|T|^2 = 2 per nonzero frequency)
static bool device_direction_staggered(const Ctx& X, int n, double delta, host::HTT& out) {
  const long NN = 1L << (3 * n);
  const int L = 3 * n + 1, N = 1 << n;
  std::vector<double> kp, km;
  host::staggered_symbols(n, kp, km);
  auto sd = X.buf(2 * (size_t)N);
  check(hipMemcpyAsync(sd->p, kp.data(), N * sizeof(cplx), hipMemcpyHostToDevice, X.s()), "symbols h2d");
  check(hipMemcpyAsync((cplx*)sd->p + N, km.data(), N * sizeof(cplx), hipMemcpyHostToDevice, X.s()),
        "symbols h2d");
  auto T = X.buf((size_t)6 * NN);
  need(X, T->p, 6 * NN - 1, "direction out");
  direction_staggered((const cplx*)sd->p, (const cplx*)sd->p + N, n, (cplx*)T->p, X.s());
  X.sync();  // the host symbol arrays are released on return
  return device_ttsvd(X, T, 3 * n, 6, delta / std::sqrt((double)(L - 1)) * std::sqrt(2.0 * (double)(NN - 1)),
                      out);
}

// The plane staggered directions (n_a, m_a), a in {x, y}: 4 x 2^(2n)
static bool device_direction_staggered2d(const Ctx& X, int n, double delta, host::HTT& out) {
  const long NN = 1L << (2 * n);
  const int L = 2 * n + 1, N = 1 << n;
  std::vector<double> kp, km;
  host::staggered_symbols(n, kp, km);
  auto sd = X.buf(2 * (size_t)N);
  check(hipMemcpyAsync(sd->p, kp.data(), N * sizeof(cplx), hipMemcpyHostToDevice, X.s()), "symbols h2d");
  check(hipMemcpyAsync((cplx*)sd->p + N, km.data(), N * sizeof(cplx), hipMemcpyHostToDevice, X.s()),
        "symbols h2d");
  auto T = X.buf((size_t)4 * NN);
  need(X, T->p, 4 * NN - 1, "direction out");
  direction_staggered2d((const cplx*)sd->p, (const cplx*)sd->p + N, n, (cplx*)T->p, X.s());
  X.sync();
  return device_ttsvd(X, T, 2 * n, 4, delta / std::sqrt((double)(L - 1)) * std::sqrt(2.0 * (double)(NN - 1)),
                      out);
}

// TT-SVD of a dense device tensor T with dims (P, 2, ..., 2) (3n binary
// indices, P slowest; complex storage, P 2^(3n) entries), right to left: the
// unfolding M (P 2^(k-1) x 2 r_k) is reduced to R by tsqr_r, R^H goes
// through the one-sided Jacobi (its left singular vectors are M's right
// singular vectors V, sorted by singular value), the rank follows the
// per-bond rule (singular values beyond rank r carry at most thr in 2-norm,
// thr = delta / sqrt(L - 1) ||T||), core k = V_r^H and M <- M V_r continues
// with the next bit.  Returns the cores on the host (r_{k-1}, d_k, r_k);
// false when a bond would need more than 160 (the Jacobi's 320 columns).
static bool device_ttsvd(const Ctx& X, BufP T, int bits, int P, double thr, host::HTT& out) {
  const long NN = 1L << bits;
  const int L = bits + 1;
  host::HTT cores(L);
  BufP M = T;
  long rows = (long)P * NN / 2;
  int rk = 1;  // rank to the right of the current core
  for (int k = L - 1; k >= 1; --k) {
    const int c = 2 * rk;
    if (c > 320) return false;
    auto R = tsqr_r(X, M, rows, c);
    auto U = X.buf((size_t)c * c);
    auto Sd = X.bufd(c);
    jacobi_any(X, 1, c, MatView{(cplx*)R->p, 1, (long)c, (long)c * c, 1},
               MatOut{(cplx*)U->p, (long)c, 1, (long)c * c}, (double*)Sd->p);
    std::vector<double> S(c);
    std::vector<cplx> Uh((size_t)c * c);
    check(hipMemcpyAsync(S.data(), Sd->p, c * sizeof(double), hipMemcpyDeviceToHost, X.s()), "S d2h");
    check(hipMemcpyAsync(Uh.data(), U->p, Uh.size() * sizeof(cplx), hipMemcpyDeviceToHost, X.s()), "U d2h");
    X.sync();
    const int r = keep_rank(S.data(), c, thr, 0);
    host::HCore& hc = cores[k];
    hc.r0 = r; hc.dout = 2; hc.din = 0; hc.r1 = rk;
    hc.v.resize((size_t)r * c);
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < c; ++j) {
        const cplx u = Uh[(size_t)j * c + i];  // V_r^H[i][j] = conj(U[j][i])
        hc.v[(size_t)i * c + j] = std::complex<double>(u.x, -u.y);
      }
    // M <- M V_r in row chunks (the GEMM grid bounds the rows per product)
    auto Mn = X.buf((size_t)rows * r);
    // rows is P times a power of two: halve the chunk while it stays at
    // least max(4096, rows / 32768) rows and divides rows
    const long target = std::max<long>(4096, rows / 32768);
    long nbt = 1;
    while (rows % (2 * nbt) == 0 && rows / (2 * nbt) >= target) nbt *= 2;
    const long ch = rows / nbt;
    G(X, (int)ch, r, c, OP_N, (cplx*)M->p, c, OP_N, (cplx*)U->p, c, (cplx*)Mn->p, r, (int)nbt,
      ch * c, 0, ch * r);
    M = Mn;
    rk = r;
    rows /= 2;
  }
  // core 0: M is (P x r_0)
  host::HCore& h0 = cores[0];
  h0.r0 = 1; h0.dout = P; h0.din = 0; h0.r1 = rk;
  std::vector<cplx> m0((size_t)P * rk);
  check(hipMemcpyAsync(m0.data(), M->p, m0.size() * sizeof(cplx), hipMemcpyDeviceToHost, X.s()), "core0 d2h");
  X.sync();
  h0.v.resize(m0.size());
  for (size_t e = 0; e < m0.size(); ++e) h0.v[e] = std::complex<double>(m0[e].x, m0[e].y);
  out = std::move(cores);
  return true;
}

// Raised stiffness operator (and the one-hot train) of a problem: the
// device TT-SVD, or the host one when a bond rank exceeds the device path.
static host::HTT stiffness_op(const Ctx& X, const uint8_t* phase, bool on_device, int n, int P,
                              const double* lame, const double* lame0, double delta, int cap,
                              host::HTT* chi, int dim = 3) {
  host::HTT t;
  if (device_chi(X, phase, on_device, dim * n, P, delta, t))
    return host::stiffness_from_chi(std::move(t), P, lame, lame0, cap, chi, nullptr, dim == 2 ? 3 : 6);
  std::vector<uint8_t> tmp;
  const uint8_t* ph = phase;
  if (on_device) {
    tmp.resize((size_t)1 << (dim * n));
    check(hipMemcpy(tmp.data(), phase, tmp.size(), hipMemcpyDeviceToHost), "phase d2h");
    ph = tmp.data();
  }
  if (dim == 2) {
    // host TT-SVD of the one-hot pixel train (bonds beyond the device path)
    const size_t NN = (size_t)1 << (2 * n);
    std::vector<double> oh((size_t)P * NN, 0.0);
    for (size_t e = 0; e < NN; ++e) {
      if (ph[e] >= P) throw std::invalid_argument("phase id out of range");
      oh[(size_t)ph[e] * NN + e] = 1.0;
    }
    std::vector<int> dims(2 * n + 1, 2);
    dims[0] = P;
    host::HTT t2 = host::tt_svd_real(oh, dims, delta, 0);
    return host::stiffness_from_chi(std::move(t2), P, lame, lame0, cap, chi, nullptr, 3);
  }
  return host::stiffness_tto(ph, n, P, lame, lame0, delta, cap, chi, nullptr);
}

// The phase array of a problem in host memory (copied from the device when
// phase_on_device is set; tmp holds the copy).
static const uint8_t* host_phase(const qtt_problem* P, std::vector<uint8_t>& tmp) {
  if (!P->phase_on_device) return P->phase;
  tmp.resize((size_t)1 << ((P->dim == 2 ? 2 : 3) * P->n));
  check(hipMemcpy(tmp.data(), P->phase, tmp.size(), hipMemcpyDeviceToHost), "phase d2h");
  return tmp.data();
}

static Ops build_ops(const Ctx& X, const qtt_problem* P, double delta) {
  Ops o;
  const int n = P->n, dim = P->dim == 2 ? 2 : 3, V = dim == 2 ? 3 : 6;
  o.S = sfft_cached(X, n, delta, dim);
  o.G = green_cached(X, n, P->lame0[0], P->lame0[1], delta, P->scheme, dim);
  host::HTT cd = stiffness_op(X, P->phase, P->phase_on_device != 0, n, P->nphase, P->lame, P->lame0,
                              delta, 0, &o.chi, dim);
  o.Cd = upload_op(X, cd);
  o.I = identity_op(X, dim * n, V);
  o.lam0 = P->lame0[0];
  o.mu0 = P->lame0[1];
  return o;
}

static void check_problem(const qtt_problem* P, const qtt_solve_opts* O) {
  if (!P || !O) throw std::invalid_argument("null problem or options");
  if (P->dim != 0 && P->dim != 2 && P->dim != 3) throw std::invalid_argument("dim must be 0, 2 or 3");
  if (P->n < 1 || P->n > (P->dim == 2 ? 12 : 10))
    throw std::invalid_argument("n out of range (1..10, plane problems 1..12)");
  if (P->nphase < 1 || P->nphase > 16) throw std::invalid_argument("nphase out of range");
  if (!P->phase || !P->lame) throw std::invalid_argument("null phase or lame");
  if (P->scheme != QTT_SCHEME_DIRECT && P->scheme != QTT_SCHEME_STAGGERED)
    throw std::invalid_argument("scheme must be QTT_SCHEME_DIRECT or QTT_SCHEME_STAGGERED");
  if (!(O->delta > 0.0) || !(O->tol >= 0.0) || O->max_iter < 0)
    throw std::invalid_argument("bad solve options");
  if (O->precision != QTT_PREC_FP64 && O->precision != QTT_PREC_FP32 && O->precision != QTT_PREC_BF16X3)
    throw std::invalid_argument("precision must be QTT_PREC_FP64, QTT_PREC_FP32 or QTT_PREC_BF16X3");
  if (O->history && O->history_len < 1) throw std::invalid_argument("history without a length");
  if (O->orth != QTT_ORTH_HOUSEHOLDER && O->orth != QTT_ORTH_CHOLQR && O->orth != QTT_ORTH_AUTO)
    throw std::invalid_argument("orth must be QTT_ORTH_HOUSEHOLDER, QTT_ORTH_CHOLQR or QTT_ORTH_AUTO");
  if (O->matvec != QTT_MV_SKETCH && O->matvec != QTT_MV_AMEN)
    throw std::invalid_argument("matvec must be QTT_MV_SKETCH or QTT_MV_AMEN");
  for (int i = 0; i < 2 * P->nphase; ++i)
    if (!std::isfinite(P->lame[i])) throw std::invalid_argument("non-finite phase modulus");
  if (!std::isfinite(P->lame0[0]) || !(P->lame0[1] > 0.0) || !(P->lame0[0] + 2.0 * P->lame0[1] > 0.0))
    throw std::invalid_argument("reference medium must be finite with mu0 > 0, lam0 + 2 mu0 > 0");
}

struct SolveOut {
  TTP eps;
  std::vector<int> ks;
  std::vector<int> iters;
  std::vector<double> res;
  int max_rank = 1;
  double disc = 0.0;
  bool converged = true;
};

static SketchOpts sk(const Ctx& X, const qtt_solve_opts* O) {
  SketchOpts s;
  s.delta = O->delta;
  s.cap = O->cap;
  s.oversample = std::max(0, O->oversample);
  s.exact = O->exact != 0;
  s.fp32 = O->precision == QTT_PREC_FP32;
  s.bf16 = O->precision == QTT_PREC_BF16X3;
  s.orth = O->orth;
  s.matvec = O->matvec;
  s.seed = O->seed * 1000003ULL + (X.c->sketch_counter++);
  return s;
}

// options for an intermediate product of the fixed-point update
// The iterate is cap-bound: a bond rank at a cap that truncates there
// (below the bond's structural rank), and the last truncation of the
// iterate discarded at least 1e-5 of it (30 times what a dropped direction
// of the range finder can carry), so the cap, not delta, sets the error.
static bool saturated(const TT& x, int cap, double last_disc) {
  if (cap <= 0 || !(last_disc >= 1e-5)) return false;
  double left = 1.0;
  for (int k = 1; k < x.L; ++k) {
    left *= x.dout[k - 1];
    double right = 1.0;
    for (int i = k; i < x.L; ++i) right *= x.dout[i];
    if (x.r[k] >= cap && std::min(left, right) > cap) return true;
  }
  return false;
}
static SketchOpts satur(SketchOpts s, bool sat) {
  s.saturated = sat;
  return s;
}

static SketchOpts ski(const Ctx& X, const qtt_solve_opts* O) {
  SketchOpts s = sk(X, O);
  // Products whose result is sketched again at once keep the sketch rank
  // (cap + oversample) instead of a truncated-SVD sweep: the next
  // contraction costs more, the skipped sweep saves more (measured at
  // 256^3, rank 64: 23.7 vs 18.2 updates/s).  Only the iterate itself is
  // truncated to the cap.
  s.no_truncate = true;
  return s;
}

// hist (host, optional): hist[k * hlen + m] = relative update of load case
// k after update m + 1 (rows of the load cases in ks only)
static SolveOut ls_loop(const Ctx& X, const Ops& ops, const qtt_problem* P, const qtt_solve_opts* O,
                        const std::vector<int>& ks, double* hist = nullptr, int hlen = 0) {
  SolveOut out;
  const int n = P->n, B = (int)ks.size();
  const int dim = P->dim == 2 ? 2 : 3, V = dim == 2 ? 3 : 6;
  out.ks = ks;
  std::vector<double> E((size_t)B * V, 0.0);
  for (int b = 0; b < B; ++b) E[(size_t)b * V + ks[b]] = 1.0;
  auto Et = const_strain(X, n, B, E.data(), V, dim);
  auto eps = Et;
  const double normE = std::pow(2.0, 0.5 * dim * n);
  out.iters.assign(B, 0);
  out.res.assign(B, INFINITY);
  std::vector<char> done(B, 0);
  int m = 0;
  double last_disc = 0.0;
  AmenSlots amen;  // warm starts of the AMEn Green products (QTT_MV_AMEN)
  while (true) {
    RoundStats st;
    // fresh sketches in every update: with the same test matrices in every
    // update the truncated map is no contraction (measured: the relative
    // update grew at 64^3 cap 64 and at 256^3 cap 64, and stalled 2.5 times
    // higher at 256^3 cap 128); fresh draws decorrelate the rounding errors
    // the products of an update whose iterate sits at the cap sketch full-rank
    // unfoldings (QTT_ORTH_AUTO); the intermediate products carry the sketch
    // rank whatever their numerical rank, so their own ranks do not tell
    const bool sat = saturated(*eps, O->cap, last_disc);
    auto tau = op_apply(X, *ops.Cd, *eps, 0, satur(ski(X, O), sat), &st);
    auto th = op_apply(X, *ops.S, *tau, 0, satur(ski(X, O), sat), &st);
    SketchOpts og = satur(ski(X, O), sat);
    og.amen = &amen;
    {
      // inexact inner products: a twentieth of the last relative update
      double last = 0.0;
      for (int b = 0; b < B; ++b)
        if (!done[b] && std::isfinite(out.res[b])) last = std::max(last, out.res[b]);
      amen.tol = m == 0 ? 1e-3 : std::min(1e-3, 0.05 * last);
    }
    auto eh = op_apply(X, *ops.G, *th, 0, og, &st);
    auto y = op_apply(X, *ops.S->adj, *eh, 0, satur(ski(X, O), sat), &st);
    auto nw = round_any(X, axpby(X, 1.0, *Et, -1.0, *y), satur(sk(X, O), sat), &st);
    out.disc = std::max(out.disc, st.rel_max());
    last_disc = st.rel_max();  // the iterate's truncation (the last rounding)
    for (int k = 1; k < nw->L; ++k) out.max_rank = std::max(out.max_rank, nw->r[k]);
    double prev = 0.0;
    for (int b = 0; b < B; ++b)
      if (!done[b]) prev = std::max(prev, out.res[b]);
    std::vector<double> dn = diff_norms(X, *nw, *eps, m == 0 ? 0.0 : prev);
    eps = nw;
    ++m;
    if (verbose()) {
      std::fprintf(stderr, "[qtthom] it %d res", m);
      for (int b = 0; b < B; ++b) std::fprintf(stderr, " %.3e", dn[b] / normE);
      std::fprintf(stderr, " rank %d disc %.2e\n", out.max_rank, out.disc);
    }
    bool all = true;
    for (int b = 0; b < B; ++b) {
      const double r = dn[b] / normE;
      if (!std::isfinite(r)) throw nan_error("NaN/Inf in the fixed-point residual");
      if (!done[b]) {
        out.iters[b] = m;
        out.res[b] = r;
        if (hist && m <= hlen) hist[(size_t)ks[b] * hlen + (m - 1)] = r;
        if (r < O->tol) done[b] = 1;
      }
      all = all && done[b];
    }
    if (all) break;
    if (m >= O->max_iter) {
      out.converged = false;
      break;
    }
    for (int b = 0; b < B; ++b)
      if (!done[b] && out.res[b] > 1e3) throw std::overflow_error("fixed point diverged");
  }
  out.eps = eps;
  return out;
}

static void ceff_from(const Ctx& X, const Ops& ops, const qtt_problem* P, const SolveOut& so,
                      double* Ceff) {
  // plane problems (3 Voigt components) fill rows and columns 0..2
  const int V = P->dim == 2 ? 3 : 6;
  auto md = mean_apply(X, *ops.Cd, *so.eps);
  auto me = mean_apply(X, *ops.I, *so.eps);
  double C0m[36];
  host::iso_voigt_dim(V, P->lame0[0], P->lame0[1], C0m);
  for (size_t b = 0; b < so.ks.size(); ++b) {
    const int k = so.ks[b];
    for (int i = 0; i < V; ++i) {
      std::complex<double> s = md[b * V + i];
      for (int j = 0; j < V; ++j) s += C0m[i * V + j] * me[b * V + j];
      Ceff[i * 6 + k] = s.real();
    }
  }
}

struct Prepared {
  int n = 0, nphase = 0, load_mask = 0, scheme = 0, dim = 0;
  std::vector<uint8_t> phase;
  std::vector<double> lame;
  double lame0[2] = {0, 0};
  double delta = 0;
  Ops ops;
  double seconds_setup = 0;
  qtt_problem problem() const {
    qtt_problem P{};
    P.n = n; P.phase = phase.data(); P.nphase = nphase; P.lame = lame.data();
    P.lame0[0] = lame0[0]; P.lame0[1] = lame0[1]; P.load_mask = load_mask;
    P.phase_on_device = 0;
    P.scheme = scheme;
    P.dim = dim;
    return P;
  }
};

static void stats_collect(qtt_ctx* c) {
  if (c->pending.empty() && c->span_used == 0) return;
  check(hipStreamSynchronize(c->stream), "stats sync");
  std::vector<unsigned long long> sp;
  if (c->span_used > 0) {
    sp.resize(2 * (size_t)c->span_used);
    check(hipMemcpyAsync(sp.data(), c->span, sp.size() * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, c->stream),
          "span copy");
    check(hipStreamSynchronize(c->stream), "span copy sync");
  }
  for (auto& r : c->pending) {
    double sec = 0.0;
    if (r.slot >= 0) {
      const unsigned long long t0 = sp[2 * (size_t)r.slot], t1 = sp[2 * (size_t)r.slot + 1];
      if (t1 < t0) throw std::logic_error("stats: span slot not written by its launch");
      sec = (double)(t1 - t0) / c->span_hz;
    } else {
      float ms = 0.f;
      check(hipEventElapsedTime(&ms, r.a, r.b), "event elapsed");
      sec = 1e-3 * ms;
      c->evfree.push_back(r.a);
      c->evfree.push_back(r.b);
    }
    c->st_calls[r.fam] += 1;
    c->st_secs[r.fam] += sec;
    c->st_flops[r.fam] += r.flops;
    c->st_bytes[r.fam] += r.bytes;
  }
  c->pending.clear();
  if (c->span_used > 0) {
    span_arm(c->span, c->span_used, c->stream);
    c->span_used = 0;
  }
}

bool Ctx::k0(unsigned long long*& span, int& slot) const {
  span = nullptr;
  slot = -1;
  if (!c->stats_on) return false;
  if (c->stats_tick++ % (unsigned long long)c->stats_stride != 0) return true;
  if (!c->span) {
    int khz = 0;
    check(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device), "wall clock rate");
    if (khz <= 0) throw std::runtime_error("stats: device reports no real-time counter rate");
    c->span_hz = 1e3 * khz;
    check(hipMalloc(&c->span, 2 * sizeof(unsigned long long) * qtt_ctx::SPAN_SLOTS), "span alloc");
    span_arm(c->span, qtt_ctx::SPAN_SLOTS, c->stream);
    c->span_used = 0;
  }
  if (c->span_used == qtt_ctx::SPAN_SLOTS) stats_collect(c);  // books and re-arms the slots
  slot = c->span_used++;
  span = c->span + 2 * (size_t)slot;
  return true;
}

}  // namespace qtt

struct qtt_prepared {
  qtt::Prepared p;
};

// ---------------------------------------------------------------------------
// Fixed device workspace of the entry point that allocates nothing
// (qtt_zqr_noalloc): one array per GPU for the life of the process.  In host
// code `scratch` names a host-side stand-in, not a device address, so host
// code only ever uses the address hipGetSymbolAddress returned for the
// device at context creation (scratch_ptr).
// ---------------------------------------------------------------------------
namespace qtt {
constexpr size_t NOALLOC_ELEMS = (size_t)QTT_ZQR_NOALLOC_MAX_ELEMS;
static __device__ __align__(256) cplx scratch[NOALLOC_ELEMS];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_addr;

// Looks up (once per device, with that device current) the device address
// of `scratch`; returns nullptr until then.
static void* scratch_setup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr)
    throw std::runtime_error(std::string("scratch symbol address: ") + hipGetErrorString(e));
  g_scratch_addr[device] = p;
  return p;
}
static void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  return it == g_scratch_addr.end() ? nullptr : it->second;
}
}  // namespace qtt

// ===========================================================================
// C ABI
// ===========================================================================
using namespace qtt;

template <class F>
static int guarded(qtt_ctx* ctx, F&& f) {
  try {
    f();
    return QTT_OK;
  } catch (const std::invalid_argument& e) {
    if (ctx) ctx->err = e.what();
    return QTT_EINVAL;
  } catch (const std::length_error& e) {
    if (ctx) ctx->err = e.what();
    return QTT_ECAPACITY;
  } catch (const std::logic_error& e) {
    if (ctx) ctx->err = e.what();
    return QTT_EHIP;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "allocation failed";
    return QTT_ENOMEM;
  } catch (const std::overflow_error& e) {
    if (ctx) ctx->err = e.what();
    return QTT_EDIVERGED;
  } catch (const nan_error& e) {
    if (ctx) ctx->err = e.what();
    return QTT_ENAN;
  } catch (const std::runtime_error& e) {
    if (ctx) ctx->err = e.what();
    return QTT_EHIP;
  } catch (...) {
    if (ctx) ctx->err = "unknown error";
    return QTT_EHIP;
  }
}
#define QTT_TRY(ctx, ...) return guarded(ctx, [&]() { __VA_ARGS__; })

extern "C" {

int qtt_create(int device, void* hip_stream, qtt_ctx** out) {
  if (!out) return QTT_EINVAL;
  *out = nullptr;
  try {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return QTT_EINVAL;
    check(hipSetDevice(device), "set device");
    (void)scratch_setup(device);  // the device's fixed workspace, once per device
    auto c = std::make_unique<qtt_ctx>();
    c->device = device;
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      check(hipStreamCreate(&c->stream), "stream create");
      c->own_stream = true;
    }
    c->pool = std::make_shared<Pool>();
    c->pool->device = device;
    *out = c.release();
    return QTT_OK;
  } catch (...) {
    return QTT_EHIP;
  }
}

int qtt_destroy(qtt_ctx* c) {
  if (!c) return QTT_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  c->ident.clear();
  delete c;  // the destructor releases the stream
  return QTT_OK;
}

const char* qtt_last_error(const qtt_ctx* c) { return c ? c->err.c_str() : "null context"; }

int qtt_sync(qtt_ctx* c) {
  if (!c) return QTT_EINVAL;
  QTT_TRY(c, check(hipStreamSynchronize(c->stream), "sync"));
}

int qtt_tt_from_host(qtt_ctx* c, int L, const int* dims, const int* ranks, int batch,
                     const double* data, qtt_tensor** out) {
  if (!c || !out || !dims || !ranks || !data || L < 1 || batch < 1) return QTT_EINVAL;
  QTT_TRY(c, {
    Ctx X{c};
    if (ranks[0] != 1 || ranks[L] != 1) throw std::invalid_argument("boundary ranks must be 1");
    std::vector<int> d(dims, dims + L), r(ranks, ranks + L + 1);
    for (int k = 0; k < L; ++k)
      if (d[k] < 1 || r[k + 1] < 1) throw std::invalid_argument("bad dims or ranks");
    auto t = new_tt(X, L, batch, d, r);
    size_t off = 0;
    for (int k = 0; k < L; ++k) {
      const size_t cnt = (size_t)batch * t->celems(k);
      check(hipMemcpyAsync(t->core[k], data + 2 * off, cnt * sizeof(cplx), hipMemcpyHostToDevice, c->stream), "h2d");
      off += cnt;
    }
    X.sync();
    *out = new qtt_tensor(*t);
  });
}

int qtt_tensor_shape(const qtt_tensor* t, int* kind, int* L, int* batch, int* dims_out,
                     int* dims_in, int* ranks) {
  if (!t) return QTT_EINVAL;
  if (kind) *kind = t->kind == 0 ? 0 : 1;
  if (L) *L = t->L;
  if (batch) *batch = t->B;
  for (int k = 0; k < t->L; ++k) {
    if (dims_out) dims_out[k] = t->dout[k];
    if (dims_in) dims_in[k] = t->din[k];
  }
  if (ranks)
    for (int k = 0; k <= t->L; ++k) ranks[k] = t->r[k];
  return QTT_OK;
}

size_t qtt_tensor_size(const qtt_tensor* t) {
  if (!t || t->kind == 2) return 0;
  size_t s = 0;
  for (int k = 0; k < t->L; ++k) {
    if (t->kind == 0) s += (size_t)t->B * t->celems(k);
    else s += (size_t)t->r[k] * t->dout[k] * t->din[k] * t->r[k + 1];
  }
  return s;
}

int qtt_tensor_to_host(qtt_ctx* c, const qtt_tensor* t, double* data, size_t capacity) {
  if (!c || !t || !data) return QTT_EINVAL;
  if (t->kind == 2) {
    c->err = "Green operator is factored; query its factors";
    return QTT_EINVAL;
  }
  if (capacity < qtt_tensor_size(t)) return QTT_ECAPACITY;
  QTT_TRY(c, {
    size_t off = 0;
    for (int k = 0; k < t->L; ++k) {
      if (t->kind == 0 || t->diag[k]) {
        const size_t cnt = (size_t)t->B * t->celems(k);
        if (t->kind == 0) {
          check(hipMemcpyAsync(data + 2 * off, t->core[k], cnt * sizeof(cplx), hipMemcpyDeviceToHost, c->stream), "d2h");
          off += cnt;
        } else {
          std::vector<std::complex<double>> tmp(cnt);
          check(hipMemcpyAsync(tmp.data(), t->core[k], cnt * sizeof(cplx), hipMemcpyDeviceToHost, c->stream), "d2h");
          check(hipStreamSynchronize(c->stream), "sync");
          const int r0 = t->r[k], d = t->dout[k], r1 = t->r[k + 1];
          const size_t full = (size_t)r0 * d * d * r1;
          std::vector<std::complex<double>> f(full, 0.0);
          for (int a = 0; a < r0; ++a)
            for (int i = 0; i < d; ++i)
              for (int b = 0; b < r1; ++b)
                f[(((size_t)a * d + i) * d + i) * r1 + b] = tmp[((size_t)a * d + i) * r1 + b];
          std::memcpy(data + 2 * off, f.data(), full * sizeof(cplx));
          off += full;
        }
      } else {
        const size_t cnt = (size_t)t->r[k] * t->dout[k] * t->din[k] * t->r[k + 1];
        check(hipMemcpyAsync(data + 2 * off, t->coreR[k], cnt * sizeof(cplx), hipMemcpyDeviceToHost, c->stream), "d2h");
        off += cnt;
      }
    }
    check(hipStreamSynchronize(c->stream), "sync");
  });
}

int qtt_tensor_destroy(qtt_tensor* t) {
  delete t;
  return QTT_OK;
}

// shape of a train from the ABI arrays (ranks[0] = ranks[L] = 1)
static void tt_spec(int L, const int* dims, const int* ranks, int batch, std::vector<int>& d,
                    std::vector<int>& r) {
  if (L < 1 || !dims || !ranks || batch < 1) throw std::invalid_argument("bad train shape");
  if (ranks[0] != 1 || ranks[L] != 1) throw std::invalid_argument("boundary ranks must be 1");
  d.assign(dims, dims + L);
  r.assign(ranks, ranks + L + 1);
  for (int k = 0; k < L; ++k)
    if (d[k] < 1 || r[k + 1] < 1) throw std::invalid_argument("bad dims or ranks");
}

int qtt_tensor_create(qtt_ctx* c, int L, const int* dims, const int* ranks, int batch,
                      qtt_tensor** out) {
  if (!c || !out) return QTT_EINVAL;
  QTT_TRY(c, {
    Ctx X{c};
    std::vector<int> d, r;
    tt_spec(L, dims, ranks, batch, d, r);
    auto t = new_tt(X, L, batch, d, r);
    for (int k = 0; k < L; ++k) ck_fill(X, t->core[k], (size_t)batch * t->celems(k), C0(), X.s());
    X.sync();
    *out = new qtt_tensor(*t);
  });
}

int qtt_tensor_wrap(qtt_ctx* c, int L, const int* dims, const int* ranks, int batch, void* dev,
                    size_t bytes, qtt_tensor** out) {
  if (!c || !out || !dev) return QTT_EINVAL;
  QTT_TRY(c, {
    std::vector<int> d, r;
    tt_spec(L, dims, ranks, batch, d, r);
    if ((uintptr_t)dev % alignof(cplx) != 0) throw std::invalid_argument("wrapped memory not 16-byte aligned");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, dev) != hipSuccess || attr.type != hipMemoryTypeDevice ||
        attr.device != c->device)
      throw std::invalid_argument("wrapped memory is not device memory of the context's device");
    auto t = std::make_shared<qtt_tensor>();
    t->kind = 0; t->L = L; t->B = batch; t->dout = d; t->din = d; t->r = r;
    t->diag.assign(L, 0);
    t->pool = c->pool;
    t->core.resize(L);
    size_t need_b = 0;
    for (int k = 0; k < L; ++k) need_b += (size_t)batch * t->celems(k) * sizeof(cplx);
    if (need_b > bytes) throw std::length_error("wrapped memory smaller than the cores");
    auto reg = std::make_shared<Buf>(c->pool, dev, need_b);
    size_t off = 0;
    for (int k = 0; k < L; ++k) {
      t->core[k] = (cplx*)((char*)dev + off);
      off += (size_t)batch * t->celems(k) * sizeof(cplx);
    }
    t->mem.push_back(reg);
    *out = new qtt_tensor(*t);
  });
}

int qtt_tensor_core(const qtt_tensor* t, int k, void** dev, size_t* bytes) {
  if (!t || !dev || t->kind != 0 || k < 0 || k >= t->L) return QTT_EINVAL;
  *dev = t->core[k];
  if (bytes) *bytes = (size_t)t->B * t->celems(k) * sizeof(cplx);
  return QTT_OK;
}

int qtt_tensor_export(qtt_ctx* c, const qtt_tensor* t, void* dev, size_t bytes) {
  if (!c || !t || !dev || t->kind != 0) return QTT_EINVAL;
  if (bytes < qtt_tensor_size(t) * sizeof(cplx)) return QTT_ECAPACITY;
  QTT_TRY(c, {
    size_t off = 0;
    for (int k = 0; k < t->L; ++k) {
      const size_t b = (size_t)t->B * t->celems(k) * sizeof(cplx);
      check(hipMemcpyAsync((char*)dev + off, t->core[k], b, hipMemcpyDeviceToDevice, c->stream), "export d2d");
      off += b;
    }
    check(hipStreamSynchronize(c->stream), "export sync");
  });
}

int qtt_const_strain(qtt_ctx* c, int n, int batch, const double* E, qtt_tensor** out) {
  if (!c || !E || !out || n < 1 || n > 10 || batch < 1) return QTT_EINVAL;
  QTT_TRY(c, {
    Ctx X{c};
    *out = new qtt_tensor(*const_strain(X, n, batch, E));
  });
}

int qtt_sfft_build(qtt_ctx* c, int n, double delta, qtt_tensor** S) {
  if (!c || !S || n < 1 || n > 10 || !(delta > 0)) return QTT_EINVAL;
  QTT_TRY(c, {
    Ctx X{c};
    *S = new qtt_tensor(*sfft_op(X, n, delta));
  });
}

int qtt_green_build(qtt_ctx* c, int n, double lam0, double mu0, double delta, qtt_tensor** Gp) {
  return qtt_green_build_scheme(c, n, lam0, mu0, delta, QTT_SCHEME_DIRECT, Gp);
}

int qtt_green_build_scheme(qtt_ctx* c, int n, double lam0, double mu0, double delta, int scheme,
                           qtt_tensor** Gp) {
  if (!c || !Gp || n < 1 || n > 9 || !(mu0 > 0) || !(lam0 + 2 * mu0 > 0) || !(delta > 0) ||
      (scheme != QTT_SCHEME_DIRECT && scheme != QTT_SCHEME_STAGGERED))
    return QTT_EINVAL;
  QTT_TRY(c, {
    Ctx X{c};
    *Gp = new qtt_tensor(*green_op(X, n, lam0, mu0, delta, scheme));
  });
}

int qtt_rank_estimate(qtt_ctx* c, const uint8_t* phase, int phase_on_device, int n, int nphase, double delta,
                      int* ranks, double* growth) {
  return qtt_rank_estimate_dim(c, phase, phase_on_device, n, nphase, delta, 3, ranks, growth);
}

int qtt_rank_estimate_dim(qtt_ctx* c, const uint8_t* phase, int phase_on_device, int n, int nphase,
                          double delta, int dim, int* ranks, double* growth) {
  if (!c || !phase || !ranks || (dim != 2 && dim != 3) || n < 2 || n > (dim == 2 ? 12 : 8) || nphase < 1 ||
      nphase > 16 || !(delta > 0))
    return QTT_EINVAL;
  QTT_TRY(c, {
    Ctx X{c};
    const long NN = 1L << (dim * n);
    const uint8_t* dph = phase;
    BufP phb;
    if (!phase_on_device) {
      phb = X.buf((size_t)(NN + 15) / 16);
      check(hipMemcpyAsync(phb->p, phase, NN, hipMemcpyHostToDevice, X.s()), "phase h2d");
      dph = (const uint8_t*)phb->p;
    }
    const long NC = NN >> dim;  // pixels or voxels one order lower
    auto cb = X.buf((size_t)(NC + 15) / 16);
    need(X, cb->p, (long)((NC + 15) / 16) - 1, "coarse out");
    coarsen_majority(dph, n, nphase, (uint8_t*)cb->p, X.s(), dim);
    host::HTT fine, coarse;
    // the device TT-SVD, or the host one where a bond exceeds its 160
    auto chi_of = [&](const uint8_t* d, int bits, host::HTT& out) {
      if (device_chi(X, d, true, bits, nphase, delta, out)) return;
      const size_t M = (size_t)1 << bits;
      std::vector<uint8_t> h(M);
      check(hipMemcpy(h.data(), d, M, hipMemcpyDeviceToHost), "phase d2h");
      std::vector<double> oh((size_t)nphase * M, 0.0);
      for (size_t e = 0; e < M; ++e) {
        if (h[e] >= nphase) throw std::invalid_argument("phase id out of range");
        oh[(size_t)h[e] * M + e] = 1.0;
      }
      std::vector<int> dims(bits + 1, 2);
      dims[0] = nphase;
      out = host::tt_svd_real(oh, dims, delta, 0);
    };
    chi_of(dph, dim * n, fine);
    chi_of((const uint8_t*)cb->p, dim * (n - 1), coarse);
    int rc = 1, rf = 1;
    for (const auto& h : coarse) rc = std::max(rc, h.r1);
    for (const auto& h : fine) rf = std::max(rf, h.r1);
    ranks[0] = rc;
    ranks[1] = rf;
    if (growth) *growth = (double)rf / rc;
  });
}

int qtt_from_voxels(qtt_ctx* c, const uint8_t* phase, int phase_on_device, int n, int nphase,
                    const double* lame, const double lame0[2], double delta, int cap,
                    qtt_tensor** Cm, qtt_tensor** chi) {
  return qtt_from_voxels_dim(c, phase, phase_on_device, n, nphase, lame, lame0, delta, cap, 3, Cm, chi);
}

int qtt_from_voxels_dim(qtt_ctx* c, const uint8_t* phase, int phase_on_device, int n, int nphase,
                        const double* lame, const double lame0[2], double delta, int cap, int dim,
                        qtt_tensor** Cm, qtt_tensor** chi) {
  if (!c || !phase || !lame || !lame0 || !Cm || (dim != 2 && dim != 3) || n < 1 || n > (dim == 2 ? 12 : 9) ||
      nphase < 1 || nphase > 16)
    return QTT_EINVAL;
  QTT_TRY(c, {
    Ctx X{c};
    host::HTT chih;
    host::HTT cd =
        stiffness_op(X, phase, phase_on_device != 0, n, nphase, lame, lame0, delta, cap, &chih, dim);
    *Cm = new qtt_tensor(*upload_op(X, cd));
    if (chi) {
      // the one-hot train as a train (kind 0, batch 1)
      std::vector<int> d, r;
      r.push_back(1);
      for (auto& cc : chih) { d.push_back(cc.dout); r.push_back(cc.r1); }
      auto t = new_tt(X, (int)chih.size(), 1, d, r);
      for (size_t k = 0; k < chih.size(); ++k)
        check(hipMemcpyAsync(t->core[k], chih[k].v.data(), chih[k].v.size() * sizeof(cplx), hipMemcpyHostToDevice, c->stream), "chi h2d");
      X.sync();
      *chi = new qtt_tensor(*t);
    }
  });
}

static int product(qtt_ctx* c, const qtt_tensor* A, const qtt_tensor* x, qtt_tensor** y, int flags,
                   double delta, int cap, uint64_t seed, bool inverse_ok) {
  if (!c || !A || !x || !y || x->kind != 0 || !(delta > 0)) return QTT_EINVAL;
  QTT_TRY(c, {
    Ctx X{c};
    const qtt_tensor* op = A;
    if (inverse_ok && (flags & QTT_INVERSE)) {
      if (!A->adj) throw std::invalid_argument("operator has no stored inverse");
      op = A->adj.get();
    }
    SketchOpts o;
    o.delta = delta;
    o.cap = cap;
    o.seed = seed;
    *y = new qtt_tensor(*op_apply(X, *op, *x, flags, o, nullptr));
  });
}

int sfft_apply(qtt_ctx* c, const qtt_tensor* S, const qtt_tensor* x, qtt_tensor** y, int flags,
               double delta, int cap, uint64_t seed) {
  return product(c, S, x, y, flags, delta, cap, seed, true);
}

int tt_hadamard(qtt_ctx* c, const qtt_tensor* A, const qtt_tensor* x, qtt_tensor** y, int flags,
                double delta, int cap, uint64_t seed) {
  if (A && A->kind != 1) return QTT_EINVAL;
  return product(c, A, x, y, flags, delta, cap, seed, false);
}

int green_apply(qtt_ctx* c, const qtt_tensor* Gm, const qtt_tensor* x, qtt_tensor** y, int flags,
                double delta, int cap, uint64_t seed) {
  if (Gm && Gm->kind != 2) return QTT_EINVAL;
  return product(c, Gm, x, y, flags, delta, cap, seed, false);
}

int tt_amen_apply(qtt_ctx* c, const qtt_tensor* A, const qtt_tensor* x, const qtt_tensor* y0,
                  const qtt_tensor* z0, double delta, int cap, int sweeps, double tol, qtt_tensor** y,
                  int* sweeps_run, double* change) {
  if (!c || !A || !x || !y0 || !z0 || !y || A->kind != 1 || x->kind != 0 || !(delta > 0) || sweeps < 1 ||
      !(tol >= 0))
    return QTT_EINVAL;
  QTT_TRY(c, {
    Ctx X{c};
    AmenInfo inf;
    *y = new qtt_tensor(*amen_apply(X, *A, *x, *y0, *z0, delta, cap, sweeps, tol, &inf));
    if (sweeps_run) *sweeps_run = inf.sweeps;
    if (change) *change = inf.change;
  });
}

int tt_round(qtt_ctx* c, qtt_tensor* x, double delta, int cap, double* discarded) {
  if (!c || !x || x->kind != 0 || !(delta >= 0)) return QTT_EINVAL;
  QTT_TRY(c, {
    Ctx X{c};
    RoundStats st;
    round_tt(X, *x, delta, cap, &st);
    if (discarded)
      for (int b = 0; b < x->B; ++b) discarded[b] = st.norm[b] > 0 ? std::sqrt(st.disc2[b]) / st.norm[b] : 0.0;
  });
}

int tt_norm(qtt_ctx* c, const qtt_tensor* x, double* out) {
  if (!c || !x || !out || x->kind != 0) return QTT_EINVAL;
  QTT_TRY(c, {
    Ctx X{c};
    auto v = tt_norms(X, *x);
    for (int b = 0; b < x->B; ++b) out[b] = v[b];
  });
}

int tt_axpby(qtt_ctx* c, double alpha, const qtt_tensor* x, double beta, const qtt_tensor* y,
             qtt_tensor** z) {
  if (!c || !x || !y || !z || x->kind != 0 || y->kind != 0) return QTT_EINVAL;
  QTT_TRY(c, {
    Ctx X{c};
    *z = new qtt_tensor(*axpby(X, alpha, *x, beta, *y));
  });
}

int tt_mean_apply(qtt_ctx* c, const qtt_tensor* A, const qtt_tensor* x, double* out) {
  if (!c || !A || !x || !out || A->kind != 1 || x->kind != 0) return QTT_EINVAL;
  QTT_TRY(c, {
    Ctx X{c};
    auto v = mean_apply(X, *A, *x);
    std::memcpy(out, v.data(), v.size() * sizeof(cplx));
  });
}

}  // extern "C"

// Runs fn(X_g, g) for g < ng concurrently, each on a sub-context with its
// own stream (default priority) and pool driven from its own host thread,
// so one group's latency-bound factorisations overlap another's
// matrix-core products.  The sub-contexts
// read the parent's buffers (operators, trains), which stay unwritten while
// the groups run, and draw sketches from disjoint counter ranges.  Kernel
// statistics are merged into the parent; the first group error is
// rethrown after every group has finished.
template <class Fn>
static void run_groups(qtt_ctx* c, int ng, Fn&& fn) {
  check(hipStreamSynchronize(c->stream), "sync before groups");  // parent work complete
  while ((int)c->subs.size() < ng) {
    auto sc = std::make_unique<qtt_ctx>();
    sc->device = c->device;
    check(hipStreamCreate(&sc->stream), "stream create");
    sc->own_stream = true;
    sc->pool = std::make_shared<Pool>();
    sc->pool->device = c->device;
    sc->parent = c;
    c->subs.push_back(std::move(sc));
  }
  std::vector<std::exception_ptr> errs(ng);
  std::vector<std::thread> th;
  for (int g = 0; g < ng; ++g) {
    qtt_ctx* sc = c->subs[g].get();
    sc->stats_on = c->stats_on;
    sc->stats_stride = c->stats_stride;
    sc->stats_tick = (unsigned long long)g;
    sc->gemm_fp32 = false;  // set per contraction by the precision scopes
    sc->gemm_bf16 = false;
    // the sketch seeds follow the parent's counter, one disjoint range per group
    sc->sketch_counter = c->sketch_counter + ((uint64_t)(g + 1) << 40);
    th.emplace_back([&, g, sc]() {
      try {
        check(hipSetDevice(sc->device), "set device");
        Ctx Xs{sc};
        fn(Xs, g);
        Xs.sync();
      } catch (...) {
        errs[g] = std::current_exception();
      }
    });
  }
  for (auto& t : th) t.join();
  c->sketch_counter += 1;
  for (int g = 0; g < ng; ++g) {
    qtt_ctx* sc = c->subs[g].get();
    stats_collect(sc);
    for (int f = 0; f < QTT_K_COUNT; ++f) {
      c->st_calls[f] += sc->st_calls[f];
      c->st_secs[f] += sc->st_secs[f];
      c->st_flops[f] += sc->st_flops[f];
      c->st_bytes[f] += sc->st_bytes[f];
      c->st_all_calls[f] += sc->st_all_calls[f];
      c->st_all_flops[f] += sc->st_all_flops[f];
      c->st_all_bytes[f] += sc->st_all_bytes[f];
      sc->st_calls[f] = sc->st_all_calls[f] = 0;
      sc->st_secs[f] = sc->st_flops[f] = sc->st_bytes[f] = sc->st_all_flops[f] = sc->st_all_bytes[f] = 0.0;
    }
  }
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
}

// The batch elements of several trains of one shape stacked into one train
// (parent pool and stream), ranks zero-padded to the largest per bond.
static TTP stack_trains(const Ctx& X, const std::vector<TTP>& parts) {
  const TT& e0 = *parts[0];
  const int L = e0.L;
  int B = 0;
  std::vector<int> r(L + 1, 1);
  for (const auto& t : parts) {
    B += t->B;
    for (int k = 0; k <= L; ++k) r[k] = std::max(r[k], t->r[k]);
  }
  auto y = new_tt(X, L, B, e0.dout, r);
  int boff = 0;
  for (const auto& tp : parts) {
    const TT& eg = *tp;
    for (int k = 0; k < L; ++k) {
      const int d = eg.dout[k], ra = eg.r[k], rb = eg.r[k + 1], Ra = r[k], Rb = r[k + 1];
      cplx* dst = y->core[k] + (long)boff * Ra * d * Rb;
      if (ra != Ra || rb != Rb) ck_fill(X, dst, (size_t)eg.B * Ra * d * Rb, C0(), X.s());
      ck_copy2d(X, eg.B, ra * d, rb, MatView{eg.core[k], (long)rb, 1, (long)ra * d * rb, 0},
                MatOut{dst, (long)Rb, 1, (long)Ra * d * Rb}, C1(), X.s());
    }
    boff += eg.B;
  }
  X.sync();  // the parts' buffers may be released on return
  return y;
}

// The load cases ks split into ng groups solved concurrently (run_groups);
// C_eff columns are written per group, the reports and strain trains merged
// in the order of ks.
static SolveOut solve_groups(qtt_ctx* c, const Prepared& pr, const qtt_problem* P,
                             const qtt_solve_opts* O, const std::vector<int>& ks, int ng,
                             double* Ceff) {
  std::vector<std::vector<int>> groups(ng);
  for (size_t i = 0; i < ks.size(); ++i) groups[i * ng / ks.size()].push_back(ks[i]);
  std::vector<SolveOut> outs(ng);
  std::vector<std::array<double, 36>> cg(ng);
  run_groups(c, ng, [&](const Ctx& Xs, int g) {
    outs[g] = ls_loop(Xs, pr.ops, P, O, groups[g], O->history, O->history_len);
    cg[g].fill(0.0);
    ceff_from(Xs, pr.ops, P, outs[g], cg[g].data());
  });
  for (int g = 0; g < ng; ++g)
    for (int k : groups[g])
      for (int i = 0; i < 6; ++i) Ceff[i * 6 + k] = cg[g][i * 6 + k];  // rows beyond V stay 0
  SolveOut so;
  so.ks = ks;
  std::vector<TTP> parts;
  for (int g = 0; g < ng; ++g) {
    so.iters.insert(so.iters.end(), outs[g].iters.begin(), outs[g].iters.end());
    so.res.insert(so.res.end(), outs[g].res.begin(), outs[g].res.end());
    so.max_rank = std::max(so.max_rank, outs[g].max_rank);
    so.disc = std::max(so.disc, outs[g].disc);
    so.converged = so.converged && outs[g].converged;
    parts.push_back(outs[g].eps);
  }
  so.eps = stack_trains(Ctx{c}, parts);
  return so;
}

static int solve_prepared(qtt_ctx* c, const Prepared& pr, const qtt_solve_opts* O, double* Ceff,
                          qtt_report* R, qtt_tensor** eps_out, double setup_seconds) {
  int status = QTT_OK;
  auto body = [&]() {
    const qtt_problem P = pr.problem();
    check_problem(&P, O);
    Ctx X{c};
    std::vector<int> ks;
    for (int k = 0; k < (P.dim == 2 ? 3 : 6); ++k)
      if (P.load_mask & (1 << k)) ks.push_back(k);
    if (ks.empty()) throw std::invalid_argument("empty load mask");
    const double t1 = now_s();
    for (int i = 0; i < 36; ++i) Ceff[i] = 0.0;
    const int ng = std::max(1, std::min<int>(O->streams, (int)ks.size()));
    if (O->history)
      for (size_t e = 0; e < (size_t)6 * O->history_len; ++e) O->history[e] = std::nan("");
    SolveOut so = ng > 1 ? solve_groups(c, pr, &P, O, ks, ng, Ceff)
                         : ls_loop(X, pr.ops, &P, O, ks, O->history, O->history_len);
    if (ng == 1) ceff_from(X, pr.ops, &P, so, Ceff);
    X.sync();
    const double t2 = now_s();
    if (R) {
      std::memset(R, 0, sizeof(*R));
      for (size_t b = 0; b < ks.size(); ++b) {
        R->iterations[ks[b]] = so.iters[b];
        R->residual[ks[b]] = so.res[b];
      }
      R->max_rank = so.max_rank;
      R->discarded = so.disc;
      R->seconds_setup = setup_seconds;
      R->seconds_solve = t2 - t1;
    }
    if (eps_out) *eps_out = new qtt_tensor(*so.eps);
    if (!so.converged) status = QTT_ENOCONV;
  };
  int rc = [&]() -> int { QTT_TRY(c, body()); }();
  if (rc == QTT_OK) rc = status;
  if (R) R->status = rc;
  return rc;
}

static Prepared make_prepared(qtt_ctx* c, const qtt_problem* P, double delta) {
  Prepared pr;
  pr.n = P->n; pr.nphase = P->nphase; pr.load_mask = P->load_mask; pr.scheme = P->scheme; pr.dim = P->dim;
  const size_t NN = (size_t)1 << ((P->dim == 2 ? 2 : 3) * P->n);
  if (P->phase_on_device) {
    pr.phase.resize(NN);
    check(hipMemcpy(pr.phase.data(), P->phase, NN, hipMemcpyDeviceToHost), "phase d2h");
  } else {
    pr.phase.assign(P->phase, P->phase + NN);
  }
  pr.lame.assign(P->lame, P->lame + 2 * P->nphase);
  pr.lame0[0] = P->lame0[0];
  pr.lame0[1] = P->lame0[1];
  pr.delta = delta;
  const double t0 = now_s();
  Ctx X{c};
  const qtt_problem Q = pr.problem();
  pr.ops = build_ops(X, &Q, delta);
  X.sync();
  pr.seconds_setup = now_s() - t0;
  return pr;
}

extern "C" {

int qtt_prepare(qtt_ctx* c, const qtt_problem* P, double delta, qtt_prepared** out) {
  if (!c || !P || !out || !P->phase || !P->lame) return QTT_EINVAL;
  *out = nullptr;
  QTT_TRY(c, {
    qtt_solve_opts o{};
    o.delta = delta;
    o.tol = 0.0;
    check_problem(P, &o);
    auto* pp = new qtt_prepared();
    try {
      pp->p = make_prepared(c, P, delta);
    } catch (...) {
      delete pp;
      throw;
    }
    *out = pp;
  });
}

int qtt_prepared_destroy(qtt_prepared* pp) {
  delete pp;
  return QTT_OK;
}

int ls_solve_prepared(qtt_ctx* c, const qtt_prepared* pp, const qtt_solve_opts* O, double* Ceff,
                      qtt_report* R, qtt_tensor** eps_out) {
  if (!c || !pp || !O || !Ceff) return QTT_EINVAL;
  return solve_prepared(c, pp->p, O, Ceff, R, eps_out, 0.0);
}

int ls_solve(qtt_ctx* c, const qtt_problem* P, const qtt_solve_opts* O, double* Ceff,
             qtt_report* R, qtt_tensor** eps_out) {
  if (!c || !Ceff || !P || !O) return QTT_EINVAL;
  Prepared pr;
  int rc = [&]() -> int {
    QTT_TRY(c, {
      check_problem(P, O);
      pr = make_prepared(c, P, O->delta);
    });
  }();
  if (rc != QTT_OK) {
    if (R) R->status = rc;
    return rc;
  }
  return solve_prepared(c, pr, O, Ceff, R, eps_out, pr.seconds_setup);
}

int qtt_zgemm(qtt_ctx* c, int opA, int opB, int M, int N, int K, const double* alpha,
              const void* A, long lda, const void* B, long ldb, const double* beta, void* Cm,
              long ldc, int batch, long sA, long sB, long sC, int path) {
  if (!c || !alpha || !beta || !A || !B || !Cm) return QTT_EINVAL;
  if (M < 0 || N < 0 || K < 1 || batch < 1 || batch > 65535 || opA < 0 || opA > 2 || opB < 0 ||
      opB > 2 || path < 0 || (path > 3 + gemm_num_tiles() && path != QTT_GEMM_PATH_BF16X3))
    return QTT_EINVAL;
  if (lda < (opA == OP_N ? K : M) || ldb < (opB == OP_N ? N : K) || ldc < N) return QTT_EINVAL;
  QTT_TRY(c, {
    GemmArgs g;
    g.M = M; g.N = N; g.K = K; g.opA = opA; g.opB = opB;
    g.A = (const cplx*)A; g.lda = lda; g.sA1 = sA; g.sA2 = 0;
    g.B = (const cplx*)B; g.ldb = ldb; g.sB1 = sB; g.sB2 = 0;
    g.C = (cplx*)Cm; g.ldc = ldc; g.sC1 = sC; g.sC2 = 0;
    g.nb1 = batch; g.nb2 = 1;
    g.alpha = make_double2(alpha[0], alpha[1]);
    g.beta = make_double2(beta[0], beta[1]);
    if (M == 0 || N == 0) return;
    BufP ws;
    g.fp32 = path == 3;
    g.bf16x3 = path == QTT_GEMM_PATH_BF16X3;
    g.tile = path >= 4 && !g.bf16x3 ? path - 4 : -1;
    const int ks = path == 1 ? 1 : gemm_ksplit(M, N, K, batch, g.fp32 || g.bf16x3, g.tile);
    if (ks > 1) {
      ws = std::make_shared<Buf>(c->pool, gemm_ws_elems(g, ks) * sizeof(cplx));
      g.ws = (cplx*)ws->p;
      g.ksplit = ks;
    }
    if (path == 0) gemm(g, c->stream);
    else if (path == 1) gemm_vector(g, c->stream);
    else if (!gemm_mfma(g, c->stream))
      throw std::invalid_argument("zgemm: shape not handled by the matrix-core kernel (needs M, N >= 16, K >= 4)");
  });
}

int qtt_zqr(qtt_ctx* c, int batch, int m, int n, const void* A, void* R, void* Qo, int path) {
  if (!c || !A || !R || batch < 1 || batch > 65535 || m < 1 || n < 1 || path < 0 || path > 6)
    return QTT_EINVAL;
  QTT_TRY(c, {
    Ctx X{c};
    const int k = std::min(m, n);
    auto ws = X.buf(qr_ws(batch, m, n));
    MatView av{(const cplx*)A, (long)n, 1, (long)m * n, 0};
    MatOut ro{(cplx*)R, (long)n, 1, (long)k * n};
    MatOut qo{(cplx*)Qo, (long)k, 1, (long)m * k};
    if (!Qo) qo = MatOut{nullptr, 0, 0, 0};
    if (path == 0) {
      qr(batch, m, n, av, ro, qo, (cplx*)ws->p, c->stream);
    } else if (path == 1) {
      qr_generic(batch, m, n, av, ro, qo, (cplx*)ws->p, c->stream);
    } else if (path == 2) {
      if (!qr_blocked(batch, m, n, av, ro, qo, (cplx*)ws->p, c->stream))
        throw std::invalid_argument("zqr: shape not covered by the blocked matrix-core kernel");
    } else if (path == 3) {
      if (!qr_fast(batch, m, n, av, ro, qo, (cplx*)ws->p, c->stream))
        throw std::invalid_argument("zqr: shape not covered by the register-resident kernels");
    } else if (path == 4) {
      if (!qr_two_col(batch, m, n, av, ro, qo, c->stream))
        throw std::invalid_argument("zqr: shape not covered by the two-column register kernel");
    } else if (path == 6) {
      if (!qr_big(batch, m, n, av, ro, qo, (cplx*)ws->p, c->stream))
        throw std::invalid_argument("zqr: shape not covered by the workspace-resident blocked kernel");
    } else {
      const bool qok = !Qo || (m >= n && n > 16 && n <= 96);
      if (!qok || !qr_one_rowblock(batch, m, n, av, ro, Qo ? (cplx*)ws->p : nullptr, c->stream))
        throw std::invalid_argument("zqr: shape not covered by the one-row-block kernel");
      if (Qo && !qr_form_q(batch, m, n, qo, (cplx*)ws->p, c->stream))
        throw std::invalid_argument("zqr: shape not covered by the matrix-core Q formation");
    }
    X.sync();  // the workspace is released on return
  });
}

int qtt_zorth(qtt_ctx* c, int batch, int m, int n, const void* A, void* Qo, int* fallback, int path) {
  if (!c || !A || !Qo || batch < 1 || batch > 65535 || m < 1 || n < 1 || path < 0 || path > 2)
    return QTT_EINVAL;
  if (!orth_ok(m, n)) {
    c->err = "qtt_zorth: " + std::to_string(m) + " x " + std::to_string(n) +
             " outside m >= n, 32 < m <= 192 for 16 < n <= 64, 32 < m <= 168 for 64 < n <= 80";
    return QTT_EINVAL;
  }
  QTT_TRY(c, {
    Ctx X{c};
    auto ws = X.buf(path != 1 ? orth_split_ws(batch, m, n) : orth_ws(batch, m, n));
    // caller-owned operands (not in the context's pool): launched directly
    const MatView av{(const cplx*)A, (long)n, 1, (long)m * n, 0};
    const MatOut qo{(cplx*)Qo, (long)n, 1, (long)m * n};
    if (path == 1) orth(batch, m, n, av, qo, (cplx*)ws->p, c->stream);
    else orth_split(batch, m, n, av, qo, (cplx*)ws->p, c->stream, path == 2);
    if (fallback)
      check(hipMemcpyAsync(fallback, ws->p, batch * sizeof(int), hipMemcpyDeviceToHost, c->stream),
            "orth flags d2h");
    X.sync();  // the workspace is released on return
  });
}

int qtt_zqr_noalloc(qtt_ctx* c, int batch, int m, int n, const void* A, void* R, void* Qo) {
  if (!c || !A || !R || batch < 1 || batch > 65535 || m < 1 || n < 1) return QTT_EINVAL;
  const size_t need_ws = qr_ws(batch, m, n);
  if (need_ws > NOALLOC_ELEMS) {
    c->err = "qtt_zqr_noalloc: batch " + std::to_string(batch) + " of " + std::to_string(m) + " x " +
             std::to_string(n) + " needs " + std::to_string(need_ws) +
             " workspace entries, more than the fixed " + std::to_string(NOALLOC_ELEMS);
    return QTT_ECAPACITY;
  }
  void* ws = scratch_ptr(c->device);
  if (!ws) {
    c->err = "qtt_zqr_noalloc: no workspace address for this device";
    return QTT_EHIP;
  }
  QTT_TRY(c, {
    const int k = std::min(m, n);
    MatView av{(const cplx*)A, (long)n, 1, (long)m * n, 0};
    MatOut ro{(cplx*)R, (long)n, 1, (long)k * n};
    MatOut qo{(cplx*)Qo, (long)k, 1, (long)m * k};
    if (!Qo) qo = MatOut{nullptr, 0, 0, 0};
    // the library's own choice of kernels (qtt_zqr path 0) on the fixed
    // workspace; no synchronisation, so the call can be captured
    qr(batch, m, n, av, ro, qo, (cplx*)ws, c->stream);
  });
}

int qtt_zjacobi(qtt_ctx* c, int batch, int n, const void* A, void* U, double* S) {
  if (!c || !A || !U || !S || batch < 1 || batch > 65535 || n < 1) return QTT_EINVAL;
  QTT_TRY(c, {
    const MatView av{(const cplx*)A, (long)n, 1, (long)n * n, 0};
    const MatOut uo{(cplx*)U, (long)n, 1, (long)n * n};
    if (n <= 96) {
      if (!jacobi_square(batch, n, av, uo, S, c->stream)) throw std::logic_error("zjacobi size");
    } else {
      if (n > 320) throw std::invalid_argument("zjacobi: n exceeds 320");
      Ctx X{c};
      auto ws = X.buf(jacobi_ws(batch, n));
      if (!jacobi_big(batch, n, av, uo, S, (cplx*)ws->p, c->stream)) throw std::logic_error("zjacobi size");
      X.sync();  // the workspace is released on return
    }
  });
}

int qtt_stats_enable(qtt_ctx* c, int on) {
  if (!c || on < 0) return QTT_EINVAL;
  c->stats_on = on != 0;
  c->stats_stride = on > 0 ? on : 1;
  c->stats_tick = 0;
  return QTT_OK;
}

int qtt_stats_get_all(qtt_ctx* c, int fam, long long* launches, double* flops, double* bytes) {
  if (!c || fam < 0 || fam >= QTT_K_COUNT) return QTT_EINVAL;
  if (launches) *launches = c->st_all_calls[fam];
  if (flops) *flops = c->st_all_flops[fam];
  if (bytes) *bytes = c->st_all_bytes[fam];
  return QTT_OK;
}

int qtt_stats_get(qtt_ctx* c, int fam, long long* launches, double* seconds, double* flops,
                  double* bytes) {
  if (!c || fam < 0 || fam >= QTT_K_COUNT) return QTT_EINVAL;
  QTT_TRY(c, {
    stats_collect(c);
    if (launches) *launches = c->st_calls[fam];
    if (seconds) *seconds = c->st_secs[fam];
    if (flops) *flops = c->st_flops[fam];
    if (bytes) *bytes = c->st_bytes[fam];
  });
}

int qtt_stats_reset(qtt_ctx* c) {
  if (!c) return QTT_EINVAL;
  QTT_TRY(c, {
    stats_collect(c);
    for (int f = 0; f < QTT_K_COUNT; ++f) {
      c->st_calls[f] = c->st_all_calls[f] = 0;
      c->st_secs[f] = c->st_flops[f] = c->st_bytes[f] = 0.0;
      c->st_all_flops[f] = c->st_all_bytes[f] = 0.0;
    }
    c->stats_tick = 0;
  });
}

}  // extern "C"

extern "C" {

// The adjoint fixed point for the load cases ks (train batch in ks order):
// w = C e_k - (C - C0) : G[w] with G = S^H Gamma S, from w = C e_k, stopped
// per case when ||w_{m+1} - w_m|| / ||C e_k|| < tol.
struct AdjOut {
  TTP w;
  std::vector<int> it;
  std::vector<double> res;
  bool conv = true;
};

// The stress fields C(x) e_k of the unit strains e_k, k in ks (batch
// element b = ks[b]): (C - C0) e_k + C0 e_k, rounded at delta / cap.
static TTP ce_trains(const Ctx& X, const Ops& ops, const qtt_problem* P, const qtt_solve_opts* O,
                     const std::vector<int>& ks) {
  const int n = P->n, B = (int)ks.size();
  const int dim = P->dim == 2 ? 2 : 3, V = dim == 2 ? 3 : 6;
  std::vector<double> E((size_t)B * V, 0.0), C0E((size_t)B * V, 0.0);
  double C0m[36];
  host::iso_voigt_dim(V, P->lame0[0], P->lame0[1], C0m);
  for (int b = 0; b < B; ++b) {
    E[(size_t)b * V + ks[b]] = 1.0;
    for (int i = 0; i < V; ++i) C0E[(size_t)b * V + i] = C0m[i * V + ks[b]];
  }
  auto Et = const_strain(X, n, B, E.data(), V, dim);
  auto C0t = const_strain(X, n, B, C0E.data(), V, dim);
  SketchOpts so = sk(X, O);
  so.exact = true;  // rank of (C - C0) E is the stiffness rank: exact
  auto dE = op_apply(X, *ops.Cd, *Et, 0, so, nullptr);
  auto Ce = axpby(X, 1.0, *dE, 1.0, *C0t);
  round_tt(X, *Ce, O->delta, O->cap, nullptr);
  return Ce;
}

static AdjOut adj_loop(const Ctx& X, const Ops& ops, const qtt_problem* P, const qtt_solve_opts* O,
                       const std::vector<int>& ks) {
  const int B = (int)ks.size();
  // C e_k trains: (C - C0) : E + C0 E
  auto Ce = ce_trains(X, ops, P, O, ks);
  std::vector<double> nCe = tt_norms(X, *Ce);
  AdjOut out;
  auto w = Ce;
  double last_disc = 0.0;
  out.it.assign(B, 0);
  out.res.assign(B, 0.0);
  std::vector<char> done(B, 0);
  int m = 0;
  AmenSlots amen;  // warm starts of the AMEn Green products (QTT_MV_AMEN)
  while (true) {
    const bool sat = saturated(*w, O->cap, last_disc);
    RoundStats st;
    auto u = op_apply(X, *ops.S, *w, 0, satur(ski(X, O), sat), nullptr);
    SketchOpts og = satur(ski(X, O), sat);
    og.amen = &amen;
    {
      double last = 0.0;
      for (int b = 0; b < B; ++b)
        if (!done[b]) last = std::max(last, out.res[b]);
      amen.tol = m == 0 ? 1e-3 : std::min(1e-3, 0.05 * last);
    }
    u = op_apply(X, *ops.G, *u, 0, og, nullptr);
    u = op_apply(X, *ops.S->adj, *u, 0, satur(ski(X, O), sat), nullptr);
    u = op_apply(X, *ops.Cd, *u, 0, satur(ski(X, O), sat), nullptr);
    auto nw = round_any(X, axpby(X, 1.0, *Ce, -1.0, *u), satur(sk(X, O), sat), &st);
    last_disc = st.rel_max();
    auto d = axpby(X, 1.0, *nw, -1.0, *w);
    auto dn = tt_norms(X, *d);
    w = nw;
    ++m;
    bool all = true;
    for (int b = 0; b < B; ++b) {
      const double r = dn[b] / std::max(nCe[b], 1e-300);
      if (!std::isfinite(r)) throw nan_error("NaN/Inf in the adjoint residual");
      if (!done[b]) {
        out.it[b] = m;
        out.res[b] = r;
        if (r < O->tol) done[b] = 1;
      }
      all = all && done[b];
    }
    if (verbose()) {
      std::fprintf(stderr, "[qtthom] adjoint it %d res", m);
      for (int b = 0; b < B; ++b) std::fprintf(stderr, " %.3e", out.res[b]);
      std::fprintf(stderr, "\n");
    }
    if (all) break;
    if (m >= O->max_iter) {
      out.conv = false;
      break;
    }
  }
  out.w = w;
  return out;
}

// Adjoint fixed point and gradient on built operators (see ls_adjoint).
static int adjoint_ops(qtt_ctx* c, const Ops& ops, const qtt_problem* P, const qtt_solve_opts* O,
                       const qtt_tensor* eps, const double* gbar, double* grad, qtt_report* R,
                       double seconds_setup) {
  int status = QTT_OK;
  auto body = [&]() {
    check_problem(P, O);
    Ctx X{c};
    const double t1 = now_s();
    const int n = P->n, np = P->nphase;
    const int dim = P->dim == 2 ? 2 : 3, V = dim == 2 ? 3 : 6;
    if (eps->kind != 0 || eps->B != V || eps->L != dim * n + 1 || eps->dout.empty() ||
        eps->dout[0] != V)
      throw std::invalid_argument("eps does not match the problem (V load cases of its grid)");
    const double NN = std::pow(2.0, (double)dim * n);
    std::vector<int> all_ks(V);
    for (int k = 0; k < V; ++k) all_ks[k] = k;
    const int ng = std::max(1, std::min<int>(O->streams, V));
    AdjOut ao;
    if (ng == 1) {
      ao = adj_loop(X, ops, P, O, all_ks);
    } else {
      std::vector<std::vector<int>> groups(ng);
      for (int i = 0; i < V; ++i) groups[i * ng / V].push_back(i);
      std::vector<AdjOut> outs(ng);
      run_groups(c, ng, [&](const Ctx& Xs, int g) { outs[g] = adj_loop(Xs, ops, P, O, groups[g]); });
      std::vector<TTP> parts;
      ao.conv = true;
      for (int g = 0; g < ng; ++g) {
        ao.it.insert(ao.it.end(), outs[g].it.begin(), outs[g].it.end());
        ao.res.insert(ao.res.end(), outs[g].res.begin(), outs[g].res.end());
        ao.conv = ao.conv && outs[g].conv;
        parts.push_back(outs[g].w);
      }
      ao.w = stack_trains(X, parts);
    }
    const auto& w = ao.w;
    const auto& it = ao.it;
    const auto& res = ao.res;
    const bool conv = ao.conv;
    // gradient: dC_kl/dtheta = <e_k . dC eps^l> - <w_k, G[dC eps^l]>
    const int nt = 2 * np;
    std::vector<double> J((size_t)V * V * nt, 0.0);
    double Dl[36], Dm[36];
    host::iso_voigt_dim(V, 1.0, 0.0, Dl);
    host::iso_voigt_dim(V, 0.0, 1.0, Dm);
    // one (phase, modulus) derivative per task; with ng > 1 the tasks run
    // on the load-case groups' sub-contexts (w and eps are only read)
    auto grad_task = [&](const Ctx& Xg, int task) {
      const int p = task / 2, t = task % 2;
      auto dC = dC_op(Xg, ops.chi, p, t == 0 ? Dl : Dm, V);
      auto v = op_apply(Xg, *dC, *eps, 0, sk(Xg, O), nullptr);   // dC : eps^l
      auto first = mean_apply(Xg, *ops.I, *v);                  // <e_k . dC eps^l>
      auto gv = op_apply(Xg, *ops.S, *v, 0, ski(Xg, O), nullptr);
      gv = op_apply(Xg, *ops.G, *gv, 0, ski(Xg, O), nullptr);
      gv = op_apply(Xg, *ops.S->adj, *gv, 0, sk(Xg, O), nullptr);
      auto gram = tt_gram(Xg, *w, *gv);                         // [k][l] sum conj(w_k) Gv_l
      for (int k = 0; k < V; ++k)
        for (int l = 0; l < V; ++l)
          J[((size_t)k * V + l) * nt + task] =
              first[(size_t)l * V + k].real() - gram[(size_t)k * V + l].real() / NN;
    };
    if (ng == 1) {
      for (int task = 0; task < nt; ++task) grad_task(X, task);
    } else {
      const int ngr = std::min(ng, nt);
      run_groups(c, ngr, [&](const Ctx& Xs, int g) {
        for (int task = g; task < nt; task += ngr) grad_task(Xs, task);
      });
    }
    if (gbar) {
      for (int t = 0; t < nt; ++t) {
        double s = 0.0;
        for (int i = 0; i < V * V; ++i) s += gbar[i] * J[(size_t)i * nt + t];
        grad[t] = s;
      }
    } else {
      std::memcpy(grad, J.data(), J.size() * sizeof(double));
    }
    X.sync();
    const double t2 = now_s();
    if (R) {
      std::memset(R, 0, sizeof(*R));
      for (int k = 0; k < V; ++k) {
        R->iterations[k] = it[k];
        R->residual[k] = res[k];
      }
      R->seconds_setup = seconds_setup;
      R->seconds_solve = t2 - t1;
    }
    if (!conv) status = QTT_ENOCONV;
  };
  int rc = [&]() -> int { QTT_TRY(c, body()); }();
  if (rc == QTT_OK) rc = status;
  if (R) R->status = rc;
  return rc;
}

int ls_adjoint(qtt_ctx* c, const qtt_problem* P, const qtt_solve_opts* O, const qtt_tensor* eps,
               const double* gbar, double* grad, qtt_report* R) {
  if (!c || !P || !O || !eps || !grad) return QTT_EINVAL;
  Ops ops;
  double setup = 0.0;
  int rc = [&]() -> int {
    QTT_TRY(c, {
      check_problem(P, O);
      Ctx X{c};
      const double t0 = now_s();
      ops = build_ops(X, P, O->delta);
      X.sync();
      setup = now_s() - t0;
    });
  }();
  if (rc != QTT_OK) {
    if (R) R->status = rc;
    return rc;
  }
  return adjoint_ops(c, ops, P, O, eps, gbar, grad, R, setup);
}

int ls_adjoint_prepared(qtt_ctx* c, const qtt_prepared* pp, const qtt_solve_opts* O,
                        const qtt_tensor* eps, const double* gbar, double* grad, qtt_report* R) {
  if (!c || !pp || !O || !eps || !grad) return QTT_EINVAL;
  const Prepared& pr = pp->p;
  qtt_problem P = pr.problem();
  return adjoint_ops(c, pr.ops, &P, O, eps, gbar, grad, R, pr.seconds_setup);
}


// Derivative of the C_eff that exactly `steps` updates of Alg. 2 return
// (no stopping test), by the reverse mode of those updates with the
// rounding held fixed:
//   eps_0 = E, eps_{m+1} = round(E - G (C - C0) eps_m),
//   C_M[k][l] = < e_k . C eps^l_M >,
//   a_M = C e_k, a_m = -(C - C0) G a_{m+1},
//   dC_M[k][l]/dtheta = < e_k . dC eps^l_M > - sum_{m < M} < G a^k_{m+1}, dC eps^l_m >.
// Every `every`-th iterate is kept (a checkpoint); the reverse sweep runs
// segment by segment from the last, recomputing a segment's iterates from
// its checkpoint with the sketches of the forward pass (seeds per update
// and product; the saturation flag of each update is kept), so that the
// recomputed iterates are the forward's.  The adjoint trains carry a sign
// that flips per update: b_M = C e_k, b_m = (C - C0) G b_{m+1}, a_m =
// (-1)^(M-m) b_m.
static int unrolled_ops(qtt_ctx* c, const Ops& ops, const qtt_problem* P, const qtt_solve_opts* O,
                        int steps, int every, const double* gbar, double* Ceff, double* grad,
                        qtt_report* R, double seconds_setup) {
  auto body = [&]() {
    check_problem(P, O);
    if (steps < 1 || steps > 100000) throw std::invalid_argument("steps must be in 1..100000");
    if (every < 0) throw std::invalid_argument("every must be >= 0 (0: keep every iterate)");
    if (O->matvec != QTT_MV_SKETCH)
      throw std::invalid_argument("the unrolled gradient takes QTT_MV_SKETCH products");
    if (!Ceff) throw std::invalid_argument("null Ceff");
    if (every == 0) every = 1;  // every iterate kept: nothing recomputed
    if (every > steps) every = steps;
    Ctx X{c};
    const double t1 = now_s();
    const int n = P->n, np = P->nphase, nt = 2 * np;
    const int dim = P->dim == 2 ? 2 : 3, V = dim == 2 ? 3 : 6;
    const double NN = std::pow(2.0, (double)dim * n);
    const double normE = std::pow(2.0, 0.5 * dim * n);
    std::vector<int> all_ks(V);
    for (int k = 0; k < V; ++k) all_ks[k] = k;
    std::vector<double> E((size_t)V * V, 0.0);
    for (int k = 0; k < V; ++k) E[(size_t)k * V + k] = 1.0;
    auto Et = const_strain(X, n, V, E.data(), V, dim);
    const unsigned long long base = O->seed * 1000003ULL + 0x5eedULL * 0x100000000ULL;
    // one update with the sketches of update m (product j: seed base + 8 m + j)
    std::vector<char> sat_at(steps, 0);
    auto opts_at = [&](int m, int j, bool inter) {
      SketchOpts so = inter ? ski(X, O) : sk(X, O);
      so.seed = base + 8ULL * (unsigned long long)m + (unsigned long long)j;
      return satur(so, sat_at[m] != 0);
    };
    auto update = [&](const TTP& eps, int m, RoundStats* st) {
      auto tau = op_apply(X, *ops.Cd, *eps, 0, opts_at(m, 0, true), st);
      auto th = op_apply(X, *ops.S, *tau, 0, opts_at(m, 1, true), st);
      auto eh = op_apply(X, *ops.G, *th, 0, opts_at(m, 2, true), st);
      auto y = op_apply(X, *ops.S->adj, *eh, 0, opts_at(m, 3, true), st);
      return round_any(X, axpby(X, 1.0, *Et, -1.0, *y), opts_at(m, 4, false), st);
    };
    // forward pass, checkpoints at m = 0, every, 2 every, ...
    std::vector<TTP> ck;
    TTP eps = Et;
    double last_disc = 0.0;
    int max_rank = 1;
    double disc = 0.0;
    std::vector<double> last_res(V, 0.0);
    for (int m = 0; m < steps; ++m) {
      if (m % every == 0) ck.push_back(eps);
      sat_at[m] = saturated(*eps, O->cap, last_disc) ? 1 : 0;
      RoundStats st;
      auto nw = update(eps, m, &st);
      last_disc = st.rel_max();
      disc = std::max(disc, last_disc);
      for (int k = 1; k < nw->L; ++k) max_rank = std::max(max_rank, nw->r[k]);
      if (m == steps - 1) {
        auto dn = tt_norms(X, *axpby(X, 1.0, *nw, -1.0, *eps));
        for (int k = 0; k < V; ++k) {
          last_res[k] = dn[k] / normE;
          if (!std::isfinite(last_res[k])) throw nan_error("NaN/Inf in the unrolled iterate");
        }
      }
      eps = nw;
    }
    for (int i = 0; i < 36; ++i) Ceff[i] = 0.0;
    {
      SolveOut so;
      so.ks = all_ks;
      so.eps = eps;
      ceff_from(X, ops, P, so, Ceff);
    }
    if (grad) {
      std::vector<double> J((size_t)V * V * nt, 0.0);
      double Dl[36], Dm[36];
      host::iso_voigt_dim(V, 1.0, 0.0, Dl);
      host::iso_voigt_dim(V, 0.0, 1.0, Dm);
      std::vector<TTP> dCs(nt);
      for (int task = 0; task < nt; ++task)
        dCs[task] = dC_op(X, ops.chi, task / 2, task % 2 == 0 ? Dl : Dm, V);
      // explicit term at the last iterate: < e_k . dC eps^l_M >
      for (int task = 0; task < nt; ++task) {
        auto v = op_apply(X, *dCs[task], *eps, 0, sk(X, O), nullptr);
        auto first = mean_apply(X, *ops.I, *v);
        for (int k = 0; k < V; ++k)
          for (int l = 0; l < V; ++l)
            J[((size_t)k * V + l) * nt + task] += first[(size_t)l * V + k].real();
      }
      auto b = ce_trains(X, ops, P, O, all_ks);
      double sgn = 1.0;
      const int nseg = (steps + every - 1) / every;
      for (int sg = nseg - 1; sg >= 0; --sg) {
        const int m0 = sg * every, m1 = std::min(steps, m0 + every);
        std::vector<TTP> seg(m1 - m0);
        seg[0] = ck[sg];
        for (int m = m0; m + 1 < m1; ++m) seg[m - m0 + 1] = update(seg[m - m0], m, nullptr);
        for (int m = m1 - 1; m >= m0; --m) {
          // g = G b_{m+1}
          auto g = op_apply(X, *ops.S, *b, 0, ski(X, O), nullptr);
          g = op_apply(X, *ops.G, *g, 0, ski(X, O), nullptr);
          g = op_apply(X, *ops.S->adj, *g, 0, sk(X, O), nullptr);
          for (int task = 0; task < nt; ++task) {
            auto v = op_apply(X, *dCs[task], *seg[m - m0], 0, sk(X, O), nullptr);
            auto gram = tt_gram(X, *g, *v);   // [k][l] sum conj(G b_k) dC eps_l
            for (int k = 0; k < V; ++k)
              for (int l = 0; l < V; ++l)
                J[((size_t)k * V + l) * nt + task] -= sgn * gram[(size_t)k * V + l].real() / NN;
          }
          if (m > 0) {
            b = op_apply(X, *ops.Cd, *g, 0, sk(X, O), nullptr);
            sgn = -sgn;
          }
        }
      }
      if (gbar) {
        for (int t = 0; t < nt; ++t) {
          double sum = 0.0;
          for (int i = 0; i < V * V; ++i) sum += gbar[i] * J[(size_t)i * nt + t];
          grad[t] = sum;
        }
      } else {
        std::memcpy(grad, J.data(), J.size() * sizeof(double));
      }
    }
    X.sync();
    const double t2 = now_s();
    if (R) {
      std::memset(R, 0, sizeof(*R));
      for (int k = 0; k < V; ++k) {
        R->iterations[k] = steps;
        R->residual[k] = last_res[k];
      }
      R->max_rank = max_rank;
      R->discarded = disc;
      R->seconds_setup = seconds_setup;
      R->seconds_solve = t2 - t1;
    }
  };
  const int rc = [&]() -> int { QTT_TRY(c, body()); }();
  if (R) R->status = rc;
  return rc;
}

int ls_unrolled(qtt_ctx* c, const qtt_problem* P, const qtt_solve_opts* O, int steps, int every,
                const double* gbar, double* Ceff, double* grad, qtt_report* R) {
  if (!c || !P || !O || !Ceff) return QTT_EINVAL;
  Ops ops;
  double setup = 0.0;
  int rc = [&]() -> int {
    QTT_TRY(c, {
      check_problem(P, O);
      Ctx X{c};
      const double t0 = now_s();
      ops = build_ops(X, P, O->delta);
      X.sync();
      setup = now_s() - t0;
    });
  }();
  if (rc != QTT_OK) {
    if (R) R->status = rc;
    return rc;
  }
  return unrolled_ops(c, ops, P, O, steps, every, gbar, Ceff, grad, R, setup);
}

int ls_unrolled_prepared(qtt_ctx* c, const qtt_prepared* pp, const qtt_solve_opts* O, int steps,
                         int every, const double* gbar, double* Ceff, double* grad, qtt_report* R) {
  if (!c || !pp || !O || !Ceff) return QTT_EINVAL;
  const Prepared& pr = pp->p;
  qtt_problem P = pr.problem();
  return unrolled_ops(c, pr.ops, &P, O, steps, every, gbar, Ceff, grad, R, pr.seconds_setup);
}

// structures per batched group: bounds the GEMM batch (6 * group * rank *
// dim must stay under the 65535 grid limit at rank 80)
static const size_t kBatchMax = 32;

// One group of structures of the same grid size solved together: the
// train batch is 6 load cases per structure, the stiffness operator holds
// one instance per structure, the SFFT and the Green factors are shared and
// the Green scalars are per structure.  The host stiffness builds (TT-SVD
// of the voxel arrays) run on parallel host threads.
static int batch_group(qtt_ctx* c, const std::vector<int>& ids, const qtt_problem* Ps,
                       const qtt_solve_opts* O, double* Ceff, qtt_report* Rs,
                       std::map<int, host::HTT>* pre = nullptr) {
  int status = QTT_OK;
  auto body = [&]() {
    const int S = (int)ids.size();
    for (int i : ids) check_problem(&Ps[i], O);
    const int n = Ps[ids[0]].n;
    const int dim = Ps[ids[0]].dim == 2 ? 2 : 3, V = dim == 2 ? 3 : 6;
    Ctx X{c};
    const double t0 = now_s();
    // per-structure stiffness operators from the device TT-SVD of each
    // voxel array (one after another on the context's stream)
    std::vector<host::HTT> cds(S);
    for (int s2 = 0; s2 < S; ++s2) {
      const qtt_problem& P = Ps[ids[s2]];
      if (pre && pre->count(ids[s2])) {
        cds[s2] = std::move((*pre)[ids[s2]]);
        continue;
      }
      host::HTT chi;
      cds[s2] = stiffness_op(X, P.phase, P.phase_on_device != 0, n, P.nphase, P.lame, P.lame0, O->delta,
                             0, &chi, dim);
    }
    Ops ops;
    ops.S = sfft_cached(X, n, O->delta, dim);
    std::vector<double> l0(S), m0(S);
    for (int s2 = 0; s2 < S; ++s2) {
      l0[s2] = Ps[ids[s2]].lame0[0];
      m0[s2] = Ps[ids[s2]].lame0[1];
    }
    ops.G = green_batch(X, n, O->delta, l0, m0, V, Ps[ids[0]].scheme, dim);
    ops.Cd = upload_op_batch(X, cds);
    ops.I = identity_op(X, dim * n, V);
    cds.clear();
    const double t1 = now_s();
    std::vector<int> ks((size_t)V * S);
    for (size_t b = 0; b < ks.size(); ++b) ks[b] = (int)(b % V);
    SolveOut so = ls_loop(X, ops, &Ps[ids[0]], O, ks);
    auto md = mean_apply(X, *ops.Cd, *so.eps);
    auto me = mean_apply(X, *ops.I, *so.eps);
    const double t2 = now_s();
    for (int s2 = 0; s2 < S; ++s2) {
      const int id = ids[s2];
      double C0m[36];
      host::iso_voigt_dim(V, Ps[id].lame0[0], Ps[id].lame0[1], C0m);
      double* Ce = Ceff + (size_t)36 * id;
      for (int i = 0; i < 36; ++i) Ce[i] = 0.0;
      bool all = true;
      for (int k = 0; k < V; ++k) {
        const size_t b = (size_t)s2 * V + k;
        for (int i = 0; i < V; ++i) {
          std::complex<double> v = md[b * V + i];
          for (int j = 0; j < V; ++j) v += C0m[i * V + j] * me[b * V + j];
          Ce[i * 6 + k] = v.real();
        }
        all = all && so.res[b] < O->tol;
      }
      if (Rs) {
        qtt_report& R = Rs[id];
        std::memset(&R, 0, sizeof(R));
        for (int k = 0; k < V; ++k) {
          R.iterations[k] = so.iters[(size_t)s2 * V + k];
          R.residual[k] = so.res[(size_t)s2 * V + k];
        }
        R.max_rank = so.max_rank;
        R.discarded = so.disc;
        R.seconds_setup = (t1 - t0) / S;
        R.seconds_solve = (t2 - t1) / S;
        R.status = all ? QTT_OK : QTT_ENOCONV;
      }
    }
    if (!so.converged) status = QTT_ENOCONV;
  };
  int rc = [&]() -> int { QTT_TRY(c, body()); }();
  if (rc == QTT_OK) rc = status;
  if (rc != QTT_OK && rc != QTT_ENOCONV && Rs)
    for (int i : ids) Rs[i].status = rc;
  return rc;
}

int qtt_batch_solve(qtt_ctx* c, int count, const qtt_problem* Ps, const qtt_solve_opts* O,
                    double* Ceff, qtt_report* Rs) {
  if (!c || !O || count < 0 || (count > 0 && (!Ps || !Ceff))) return QTT_EINVAL;
  // structures with all six load cases are solved together, grouped by
  // grid size and Green scheme, at most kBatchMax per group; the others one
  // by one
  // (key: grid size, dimension and scheme; plane problems need all three
  // of their load cases, 3D ones all six)
  std::map<std::pair<int, int>, std::vector<int>> groups;
  std::vector<int> single;
  for (int i = 0; i < count; ++i) {
    const bool plane = Ps[i].dim == 2;
    const int full = plane ? 0x7 : 0x3F;
    if ((Ps[i].load_mask & full) == full && Ps[i].n >= 1 && Ps[i].n <= (plane ? 12 : 10))
      groups[std::make_pair(Ps[i].n * 4 + (plane ? 2 : 3), Ps[i].scheme)].push_back(i);
    else
      single.push_back(i);
  }
  int worst = QTT_OK;
  auto note = [&](int rc) {
    if (rc != QTT_OK && (worst == QTT_OK || worst == QTT_ENOCONV)) worst = rc;
  };
  // rank buckets: the stiffness operators are built first and each group
  // splits by the power-of-two bucket of its structures' largest one-hot
  // bond rank (the geometry rank of Sec. 5.2), so the padded ranks of a
  // batch are alike
  std::map<int, host::HTT> pre;
  if (O->rank_buckets) {
    std::map<std::pair<int, int>, std::vector<int>> split;
    int rc = [&]() -> int {
      QTT_TRY(c, {
        Ctx X{c};
        for (auto& gr : groups)
          for (int i : gr.second) {
            const qtt_problem& P = Ps[i];
            check_problem(&P, O);
            host::HTT chi;
            pre[i] = stiffness_op(X, P.phase, P.phase_on_device != 0, P.n, P.nphase, P.lame, P.lame0, O->delta,
                                  0, &chi, P.dim == 2 ? 2 : 3);
            int r = 1;
            for (const auto& h : pre[i]) r = std::max(r, h.r1);
            int b = 0;
            while ((1 << b) < r) ++b;
            // key: grid size, dimension and scheme in the first entry,
            // bucket second
            split[std::make_pair(gr.first.first * 4 + gr.first.second, b)].push_back(i);
          }
      });
    }();
    if (rc != QTT_OK) return rc;
    groups.clear();
    for (auto& sp : split) groups[sp.first] = sp.second;
  }
  for (auto& gr : groups) {
    const std::vector<int>& ids = gr.second;
    for (size_t a = 0; a < ids.size(); a += kBatchMax) {
      std::vector<int> chunk(ids.begin() + a, ids.begin() + std::min(ids.size(), a + kBatchMax));
      const int rc = batch_group(c, chunk, Ps, O, Ceff, Rs, &pre);
      note(rc);
      if (rc != QTT_OK && rc != QTT_ENOCONV) return rc;
    }
  }
  for (int i : single) {
    const int rc = ls_solve(c, &Ps[i], O, Ceff + (size_t)36 * i, Rs ? &Rs[i] : nullptr, nullptr);
    note(rc);
    if (rc != QTT_OK && rc != QTT_ENOCONV) return rc;
  }
  return worst;
}

}  // extern "C"
