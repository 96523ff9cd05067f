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

}  // namespace dev
}  // namespace qtt
