// Device helpers shared by the formal-solution kernels of the library
// (nlte_residual.hip, nlte_velocity.hip): the piecewise-linear segment
// coefficients of Appendix A.1 and the per-wave LDS staging of depth-
// contiguous outputs.  Not part of the public ABI.
#pragma once

#include "nlte_internal.h"

namespace nlte {

// ---------------------------------------------------------------------------
// piecewise-linear coefficients (Appendix A.1)
// ---------------------------------------------------------------------------
// e = exp(-x), a = 1 - (1 - e)/x, b = (1 - e)/x - e.  The closed forms cancel
// at small x; below a switch point a and b come from their Taylor series
//   a/x = sum_{m>=1} (-1)^{m+1} x^{m-1} / (m+1)!,
//   b/x = sum_{m>=1} (-1)^{m+1} m x^{m-1} / (m+1)!.
//   FP64: switch at x = 0.1 (series truncation below 1e-20 relative).
//   FP32: switch at x = 0.3 with 6 terms; the worst relative error of a over
//   all x is then 8e-7 (of q = 1 - e 1.1e-7), set by the closed form's
//   cancellation just above the switch.
constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }
constexpr double ser_a(int m) { return ((m & 1) ? 1.0 : -1.0) / fact(m + 1); }
constexpr double ser_b(int m) { return ((m & 1) ? 1.0 : -1.0) * m / fact(m + 1); }

// Explicit fused multiply-adds on the path to J: the F-only and the Newton
// instantiations of the formal solution must produce bit-identical J (a
// finite-difference product subtracts one from the other), so no step may be
// left to the compiler's contraction choices.
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename R, int m, int M>
__device__ __forceinline__ void horner_ab(R x, R& pa, R& pb) {
  constexpr R ca = (R)ser_a(m), cb = (R)ser_b(m);
  if constexpr (m == M) {
    pa = ca;
    pb = cb;
  } else {
    horner_ab<R, m + 1, M>(x, pa, pb);
    pa = fmar(pa, x, ca);
    pb = fmar(pb, x, cb);
  }
}

template <typename R, int m, int M>
__device__ __forceinline__ R horner_a(R x) {
  constexpr R c = (R)ser_a(m);
  if constexpr (m == M)
    return c;
  else
    return fmar(horner_a<R, m + 1, M>(x), x, c);
}

// Below kSwitch the depth recursion takes a/x from its first kTerms series
// terms (kTermsAB for the pair a, b of the depth-parallel variant).
template <typename R> struct PL;
template <> struct PL<double> {
  static constexpr double kSwitch = 0.1;
  static constexpr int kTerms = 11;
  static constexpr int kTermsAB = 13;
  static __device__ __forceinline__ double ex(double x) { return exp(-x); }
  static __device__ __forceinline__ double div(double p, double q) { return p / q; }
};
template <> struct PL<float> {
  static constexpr float kSwitch = 0.3f;
  static constexpr int kTerms = 6;
  static constexpr int kTermsAB = 6;
  static __device__ __forceinline__ float ex(float x) { return __expf(-x); }
  static __device__ __forceinline__ float div(float p, float q) {
    return p * __builtin_amdgcn_rcpf(q);
  }
};

// Depth recursion of the piecewise-linear scheme (Appendix A.1), written as
//   I <- e I + q S_up + a (S - S_up),   q = 1 - e = a + b,
// of whose three terms e I and q S_up are never negative and the last is at
// most half their sum in size, so no step cancels (S - S_up is shared by the
// angles).  Below kSwitch a = x (a/x) from the series of a/x, q = x (1 - a)
// and e = 1 - q, all to relative accuracy; above, e is the exponential,
// q = 1 - e and a = 1 - q/x with 1/x = rb mu2 (rb = 1/base shared by the
// angles, mu2 = 2 mu).  With PM also b/x for the intensity derivatives.
// The side is chosen per wave: a wave whose lanes all fall on one side runs
// that side only, a mixed wave runs both and selects per lane (the same bits
// either way).
template <typename R, bool PM>
__device__ __forceinline__ void seg_series(R x, R& e, R& q, R& a, R& bx) {
  const R pa = horner_a<R, 1, PL<R>::kTerms>(x);
  a = pa * x;
  q = fmar(-x, a, x);
  e = (R)1 - q;
  if (PM) bx = ((R)1 - a) - pa;
}
template <typename R, bool PM>
__device__ __forceinline__ void seg_exp(R x, R rb, R mu2, R& e, R& q, R& a, R& bx) {
  e = PL<R>::ex(x);
  q = (R)1 - e;
  const R rx = rb * mu2;
  a = fmar(-q, rx, (R)1);
  if (PM) bx = (q * rx - e) * rx;
}
template <typename R, bool PM>
__device__ __forceinline__ void seg_coef(R x, R rb, R mu2, R& e, R& q, R& a, R& bx) {
  const bool small = x < PL<R>::kSwitch;
  const unsigned long long vote = __builtin_amdgcn_ballot_w64(small);
  if (vote == __builtin_amdgcn_read_exec()) {
    seg_series<R, PM>(x, e, q, a, bx);
  } else {
    seg_exp<R, PM>(x, rb, mu2, e, q, a, bx);
    if (vote != 0) {
      R es, qs, as, bs;
      seg_series<R, PM>(x, es, qs, as, bs);
      e = small ? es : e;
      q = small ? qs : q;
      a = small ? as : a;
      if (PM) bx = small ? bs : bx;
    }
  }
}

// Depth-contiguous outputs ([nu][k]) of one wave leave through a per-wave LDS
// tile of KF depths: each depth step parks its 64 values in a row of the
// tile, and every KF depths the tile is written out as 64/KF-frequency x
// KF-depth blocks, so a store instruction touches KF-value runs of a few rows
// instead of 64 scattered values.  The tile is private to the wave; the
// wavefront-scope fences order its LDS writes and reads across lanes.
template <int KF>
__device__ __forceinline__ void stage_put(double* tile, int k, int lane, double v) {
  tile[(k % KF) * kWave + lane] = v;
}

template <int KF, typename TO>
__device__ __forceinline__ void stage_flush(const double* tile, TO* __restrict__ out, int k0,
                                            int nz, int zp, int f0, int nnu, int lane) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  constexpr int FS = kWave / KF;  // frequencies per store instruction
  const int kk = lane % KF, fs = lane / KF;
  const int k = k0 + kk;
#pragma unroll
  for (int i = 0; i < KF; ++i) {
    const int fl = i * FS + fs;
    const double v = tile[kk * kWave + fl];
    if (k < nz && f0 + fl < nnu) stg(out + (size_t)(f0 + fl) * zp + k, (TO)v);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace nlte
