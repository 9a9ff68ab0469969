// Double-double (compensated) accumulation primitives for gfx950.
//
// The outer sum of the permanent formulas runs over 2^(n-1) (BB/FG) or 2^n
// (Ryser) terms with heavy cancellation; the paper's precision study (the
// Supplementary "Analysis of the Precision Issue" and the error tables) shows
// how plain binary64 accumulation loses digits.  Here each lane keeps its sum
// as an unevaluated pair (hi, lo) per real component:
//   * TwoSum (Knuth): s = fl(a+b) and the exact error e = a + b - s, six adds,
//     no branch, exact for any ordering of |a|, |b|;
//   * FastTwoSum (Dekker): same with |a| >= |b| known, three adds.
// Sums are folded into hi with TwoSum and the errors collected in lo (the
// "cascaded" compensated sum); pairs are combined with a TwoSum of the highs
// followed by a FastTwoSum renormalisation.
//
// These routines contain no multiplications, so floating-point contraction
// cannot alter them; the library is built without fast-math so that the
// compiler may not reassociate them.
#pragma once
#include <hip/hip_runtime.h>

namespace ph {

struct dd2 {        // (hi, lo) for the real and the imaginary part
  double hr, lr, hi, li;
};

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void fast_two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  e = b - (s - a);
}

// acc += x (x a plain complex value), compensated.
__device__ __forceinline__ void dd_accumulate(dd2& acc, double xr, double xi) {
  double s, e;
  two_sum(acc.hr, xr, s, e);
  acc.hr = s;
  acc.lr += e;
  two_sum(acc.hi, xi, s, e);
  acc.hi = s;
  acc.li += e;
}

// a + b for two double-double values (per component), renormalised.
__device__ __forceinline__ dd2 dd_add(const dd2& a, const dd2& b) {
  dd2 r;
  double s, e;
  two_sum(a.hr, b.hr, s, e);
  e += a.lr + b.lr;
  fast_two_sum(s, e, r.hr, r.lr);
  two_sum(a.hi, b.hi, s, e);
  e += a.li + b.li;
  fast_two_sum(s, e, r.hi, r.li);
  return r;
}

}  // namespace ph
