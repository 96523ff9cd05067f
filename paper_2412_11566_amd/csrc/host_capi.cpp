// Host-only entry points of the operator builders (no GPU needed).  Built
// into libqtthom_host.so so that the host construction of the SFFT, Green
// and stiffness operators can be checked on machines without a GPU.  The
// GPU library uploads exactly these host results.
#include "host_ops.h"

#include <cstring>
#include <exception>

using namespace qtt::host;

namespace {

// full cores (r0, dout, din, r1); diagonal and TT cores expanded to
// (r0, d, d, r1) when `expand`, else written as stored.
int dump(const HTT& t, int* ranks, int* dout, int* din, double* data, size_t cap) {
  size_t off = 0;
  ranks[0] = t.empty() ? 1 : t[0].r0;
  for (size_t k = 0; k < t.size(); ++k) {
    const HCore& c = t[k];
    ranks[k + 1] = c.r1;
    if (dout) dout[k] = c.dout;
    if (din) din[k] = c.din == 0 ? c.dout : c.din;
    const int d = c.dout, e = c.din == 0 ? c.dout : c.din;
    const size_t cnt = (size_t)c.r0 * d * e * c.r1;
    if (off + cnt > cap) return -3;
    std::complex<double>* out = reinterpret_cast<std::complex<double>*>(data) + off;
    std::memset((void*)out, 0, cnt * sizeof(std::complex<double>));
    for (int a = 0; a < c.r0; ++a)
      for (int o = 0; o < d; ++o)
        for (int i = 0; i < e; ++i)
          for (int b = 0; b < c.r1; ++b) {
            std::complex<double> v;
            if (c.din == 0) {
              if (o != i) continue;
              v = c.v[((size_t)a * d + o) * c.r1 + b];
            } else {
              v = c.v[(((size_t)a * d + o) * e + i) * c.r1 + b];
            }
            out[(((size_t)a * d + o) * e + i) * c.r1 + b] = v;
          }
    off += cnt;
  }
  return (int)t.size();
}

}  // namespace

extern "C" {

// Reduced QFT TTO Q_n; returns the number of cores or a negative code.
int qtt_host_qn_tto(int n, double delta, int* ranks, double* data, size_t cap) {
  try {
    return dump(qn_tto(n, delta), ranks, nullptr, nullptr, data, cap);
  } catch (const std::exception&) {
    return -1;
  }
}

// which: 0 = U, 1 = Sd, 2 = P, 3 = E (bounded Green factors).
// consts[0] = 1/(2 mu0), consts[1] = (lam0 + mu0) / (2 mu0 (lam0 + 2 mu0)).
int qtt_host_green(int n, double lam0, double mu0, double delta, int which, int* ranks,
                   int* dout, int* din, double* data, size_t cap, double* consts) {
  try {
    GreenFactors g = green_factors(n, lam0, mu0, delta);
    if (consts) {
      consts[0] = g.inv_2mu0;
      consts[1] = g.half_c;
    }
    const HTT& t = which == 0 ? g.U : (which == 1 ? g.Sd : (which == 2 ? g.P : g.E));
    return dump(t, ranks, dout, din, data, cap);
  } catch (const std::exception&) {
    return -1;
  }
}

int qtt_host_stiffness(const uint8_t* phase, int n, int nphase, const double* lame,
                       const double* lame0, double delta, int* ranks, int* dout, int* din,
                       double* data, size_t cap) {
  try {
    return dump(stiffness_tto(phase, n, nphase, lame, lame0, delta, 0, nullptr, nullptr), ranks,
                dout, din, data, cap);
  } catch (const std::exception&) {
    return -1;
  }
}

}  // extern "C"
