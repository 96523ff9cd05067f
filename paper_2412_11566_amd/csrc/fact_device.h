// Complex-arithmetic device helpers shared by the factorisation kernels.
#pragma once

#include "qtt_internal.h"

namespace qtt {
namespace dev {

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ cplx cdotc(cplx a, cplx b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double cabs2(cplx a) { return a.x * a.x + a.y * a.y; }
// value select (a ternary between two lvalues of a struct type selects an
// address, which pushes register arrays into scratch memory)
__device__ __forceinline__ cplx csel(bool c, cplx a, cplx b) {
  return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}
// p += conj(x) * a and a -= f * v as four fused multiply-adds each
__device__ __forceinline__ void cdot_acc(cplx& p, cplx x, cplx a) {
  p.x = fma(x.x, a.x, p.x);
  p.x = fma(x.y, a.y, p.x);
  p.y = fma(x.x, a.y, p.y);
  p.y = fma(-x.y, a.x, p.y);
}
__device__ __forceinline__ void caxpy_sub(cplx& a, cplx f, cplx v) {
  a.x = fma(-f.x, v.x, a.x);
  a.x = fma(f.y, v.y, a.x);
  a.y = fma(-f.x, v.y, a.y);
  a.y = fma(-f.y, v.x, a.y);
}

__device__ __forceinline__ cplx ldv(const MatView& v, long b, long i, long j) {
  cplx a = v.base[b * v.sb + i * v.rs + j * v.cs];
  if (v.conj) a.y = -a.y;
  return a;
}

// 1 / x from the hardware estimate and one Newton step (x normal)
__device__ __forceinline__ double rcp_nt(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// 1 / sqrt(x) and sqrt(x) from the hardware estimate and one Newton step
// (x normal, positive)
__device__ __forceinline__ double rsq_nt(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  return fma(0.5 * r, fma(-x * r, r, 1.0), r);
}
__device__ __forceinline__ double sqrt_nt(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  const double q0 = x * r;
  return fma(fma(-q0, q0, x), 0.5 * r, q0);
}

// Householder reflector of a column with leading entry al and squared norm
// s of the entries below it, H = I - tau v v^H with v = [1; x inv] and
// H^H [al; x] = [beta; 0]:
//   beta = -sign(Re al) sqrt(|al|^2 + s),  tau = (beta - al) / beta,
//   inv = 1 / (al - beta);
// the identity (tau = 0) for a column already zero below the diagonal or
// of squared norm below QR_TINY (beta and |al - beta| then stay far from
// the bottom of the double range).  Square root and reciprocals come from
// the hardware estimates with one Newton step each: the compiler's
// correctly rounded expansions form a long dependent chain, and this chain
// sits on the critical path of every elimination step.
__device__ __forceinline__ void householder(cplx al, double s, cplx& tau, cplx& inv, double& beta) {
  const double t = cabs2(al) + s;
  if ((s == 0.0 && al.y == 0.0) || t < QR_TINY) {
    tau = make_double2(0.0, 0.0);
    inv = make_double2(0.0, 0.0);
    beta = al.x;
    return;
  }
  beta = -copysign(sqrt_nt(t), al.x);
  const double rb = rcp_nt(beta);
  const cplx d = make_double2(al.x - beta, al.y);
  const double rdd = rcp_nt(cabs2(d));
  tau = make_double2((beta - al.x) * rb, -al.y * rb);
  inv = make_double2(d.x * rdd, -d.y * rdd);
}

}  // namespace dev
}  // namespace qtt
