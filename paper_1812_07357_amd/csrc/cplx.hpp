// Complex arithmetic and fully unrolled small DFTs in registers (gfx950).
//
// Every small transform here is a compile-time sized DFT
//   X[u] = sum_t x[t] exp(s 2 pi i t u / R),  s = -1 forward, +1 inverse,
// evaluated on values held in registers.  Odd prime sizes use the direct
// symmetric form; composite sizes are split Cooley-Tukey style (R = P * Q)
// with the inner twiddles folded to compile-time constants.  The constants
// are produced by constexpr Taylor series (range-reduced), so nothing is
// evaluated at run time.
#pragma once

#include <hip/hip_runtime.h>

#define PSATD_HD __host__ __device__

namespace psatd {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
PSATD_HD __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
PSATD_HD __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename T>
PSATD_HD __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
PSATD_HD __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
PSATD_HD __forceinline__ cx<T> cconj(cx<T> a) { return {a.re, -a.im}; }
template <typename T>
PSATD_HD __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
// multiply by s*i, s = -1 (forward) or +1 (inverse)
template <int S, typename T>
PSATD_HD __forceinline__ cx<T> mul_si(cx<T> a) {
  if constexpr (S < 0) return {a.im, -a.re};
  else return {-a.im, a.re};
}

// x * c for a compile-time constant c.  In FP32 the constant is carried as an
// unevaluated sum hi + lo of two floats, so that the product is as accurate as
// with an exact constant: a transform applied every time step with rounded
// constants would repeat the same rounding error each step and let it add up
// coherently, while rounding of the data itself varies from step to step.
PSATD_HD __forceinline__ float mulc(float x, double c) {
  const float hi = (float)c;
  const float lo = (float)(c - (double)hi);
  return fmaf(x, hi, x * lo);
}
PSATD_HD __forceinline__ double mulc(double x, double c) { return x * c; }
// a + x * c
PSATD_HD __forceinline__ float fmac(float x, double c, float a) {
  const float hi = (float)c;
  const float lo = (float)(c - (double)hi);
  return fmaf(x, hi, fmaf(x, lo, a));
}
PSATD_HD __forceinline__ double fmac(double x, double c, double a) { return fma(x, c, a); }

// Run-time twiddle w = exp(-2 pi i m / n): FP32 tables hold w as hi + lo pairs.
template <typename T>
struct Tw;
template <>
struct Tw<float> {
  cx<float> hi, lo;
};
template <>
struct Tw<double> {
  cx<double> hi;
};
// v * w (S < 0, forward) or v * conj(w) (S > 0, inverse)
template <int S>
PSATD_HD __forceinline__ cx<float> twmul(cx<float> v, const Tw<float>& w) {
  const float hr = w.hi.re, lr = w.lo.re;
  const float hi = (S < 0) ? w.hi.im : -w.hi.im;
  const float li = (S < 0) ? w.lo.im : -w.lo.im;
  const float cr = v.re * lr - v.im * li;
  const float ci = v.re * li + v.im * lr;
  return {fmaf(v.re, hr, fmaf(-v.im, hi, cr)), fmaf(v.re, hi, fmaf(v.im, hr, ci))};
}
template <int S>
PSATD_HD __forceinline__ cx<double> twmul(cx<double> v, const Tw<double>& w) {
  return (S < 0) ? cmul(v, w.hi) : cmulc(v, w.hi);
}

// ------------------------------------------------------------------ constexpr trig
namespace ce {
constexpr double kPi = 3.14159265358979323846264338327950288;

// sin(x) and cos(x) for |x| <= pi/4 by Taylor series (error < 1e-17).
constexpr double sin_small(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int n = 1; n < 12; ++n) {
    term *= -x2 / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double cos_small(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int n = 1; n < 12; ++n) {
    term *= -x2 / double((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}
// cos(2 pi num / den) and sin(2 pi num / den) with exact octant reduction in integers.
struct cs {
  double c, s;
};
constexpr cs unit_root(long num, long den) {
  long m = num % den;
  if (m < 0) m += den;
  // angle = 2 pi m / den = (pi/4) * (8 m / den); octant q = floor(8m/den)
  long q = (8 * m) / den;
  long rem = 8 * m - q * den;                  // in [0, den)
  double r = (kPi / 4.0) * double(rem) / double(den);  // in [0, pi/4)
  double c0 = cos_small(r), s0 = sin_small(r);
  double cr = cos_small(kPi / 4.0 - r), sr = sin_small(kPi / 4.0 - r);
  switch (q) {
    case 0: return {c0, s0};
    case 1: return {sr, cr};
    case 2: return {-s0, c0};
    case 3: return {-cr, sr};
    case 4: return {-c0, -s0};
    case 5: return {-sr, -cr};
    case 6: return {s0, -c0};
    default: return {cr, -sr};
  }
}
}  // namespace ce

// twiddle exp(S * 2 pi i * e / N) as compile-time constants
template <int S, int E, int N>
struct tw_const {
  static constexpr ce::cs v = ce::unit_root(long(E), long(N));
  static constexpr double c = v.c;
  static constexpr double s = (S < 0 ? -v.s : v.s);
};

// x * exp(S 2 pi i E / N) with trivial angles done without multiplies
template <int S, int E, int N, typename T>
PSATD_HD __forceinline__ cx<T> twiddle_const(cx<T> x) {
  constexpr int e = ((E % N) + N) % N;
  if constexpr (e == 0) {
    return x;
  } else if constexpr (2 * e == N) {
    return {-x.re, -x.im};
  } else if constexpr (4 * e == N) {
    return mul_si<S>(x);
  } else if constexpr (4 * e == 3 * N) {
    return mul_si<-S>(x);
  } else if constexpr (8 * e == N || 8 * e == 3 * N || 8 * e == 5 * N || 8 * e == 7 * N) {
    constexpr double h = 0.70710678118654752440084436210484904;
    constexpr double c = tw_const<S, e, N>::c, s = tw_const<S, e, N>::s;
    constexpr T sc = T(c > 0 ? 1 : -1), ss = T(s > 0 ? 1 : -1);
    return {mulc(sc * x.re - ss * x.im, h), mulc(sc * x.im + ss * x.re, h)};
  } else {
    constexpr double c = tw_const<S, e, N>::c, s = tw_const<S, e, N>::s;
    return {fmac(x.re, c, mulc(-x.im, s)), fmac(x.im, c, mulc(x.re, s))};
  }
}

// ------------------------------------------------------------------ small DFTs
template <int R>
struct smallest_factor {
  static constexpr int v = (R % 4 == 0) ? 4
                           : (R % 2 == 0 && R > 2) ? 2
                           : (R % 3 == 0 && R > 3) ? 3
                           : (R % 5 == 0 && R > 5) ? 5
                           : (R % 7 == 0 && R > 7) ? 7
                                                   : R;
};

template <int R, int S, typename T>
struct dft;

// Direct DFT for an odd size R using the x[t] +- x[R-t] symmetry:
//   X[u] = x0 + sum_t cos(2 pi t u / R) (x[t] + x[R-t]) + S i sin(2 pi t u / R) (x[t] - x[R-t])
// and X[R-u] the same with the sine part negated.  Constants are template immediates.
template <int R, int U, int TT, typename T>
struct odd_acc {
  static PSATD_HD __forceinline__ void run(cx<T>& a, cx<T>& b, const cx<T>* sp, const cx<T>* sm) {
    if constexpr (TT <= (R - 1) / 2) {
      constexpr double c = tw_const<1, U * TT, R>::c;
      constexpr double s = tw_const<1, U * TT, R>::s;
      a.re = fmac(sp[TT].re, c, a.re);
      a.im = fmac(sp[TT].im, c, a.im);
      b.re = fmac(sm[TT].re, s, b.re);
      b.im = fmac(sm[TT].im, s, b.im);
      odd_acc<R, U, TT + 1, T>::run(a, b, sp, sm);
    }
  }
};
template <int R, int S, int U, typename T>
struct odd_out {
  static PSATD_HD __forceinline__ void run(cx<T>* out, cx<T> x0, const cx<T>* sp, const cx<T>* sm) {
    if constexpr (U <= (R - 1) / 2) {
      cx<T> a = x0;
      cx<T> b = {T(0), T(0)};
      odd_acc<R, U, 1, T>::run(a, b, sp, sm);
      cx<T> ib = mul_si<S>(b);
      out[U] = cadd(a, ib);
      out[R - U] = csub(a, ib);
      odd_out<R, S, U + 1, T>::run(out, x0, sp, sm);
    }
  }
};
template <int R, int S, typename T>
PSATD_HD __forceinline__ void dft_odd(cx<T>* x) {
  constexpr int H = (R - 1) / 2;
  cx<T> sp[H + 1], sm[H + 1];
#pragma unroll
  for (int t = 1; t <= H; ++t) {
    sp[t] = cadd(x[t], x[R - t]);
    sm[t] = csub(x[t], x[R - t]);
  }
  cx<T> x0 = x[0];
  cx<T> dc = x0;
#pragma unroll
  for (int t = 1; t <= H; ++t) dc = cadd(dc, sp[t]);
  cx<T> out[R];
  out[0] = dc;
  odd_out<R, S, 1, T>::run(out, x0, sp, sm);
#pragma unroll
  for (int u = 0; u < R; ++u) x[u] = out[u];
}

// Generic: prime sizes go to dft_odd (or the radix-2 butterfly); composite sizes split R = P*Q.
template <int R, int S, typename T>
struct dft {
  static PSATD_HD __forceinline__ void run(cx<T>* x) {
    constexpr int P = smallest_factor<R>::v;
    if constexpr (P == R) {
      if constexpr (R == 1) {
      } else if constexpr (R == 2) {
        cx<T> a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
      } else if constexpr (R == 4) {
        cx<T> a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
        cx<T> b0 = cadd(x[1], x[3]), b1 = mul_si<S>(csub(x[1], x[3]));
        x[0] = cadd(a0, b0);
        x[2] = csub(a0, b0);
        x[1] = cadd(a1, b1);
        x[3] = csub(a1, b1);
      } else {
        dft_odd<R, S, T>(x);
      }
    } else {
      // R = P * Q; input n = Q n1 + n2, output k = k1 + P k2.
      cx<T> y[R];
      split_stage<0>(x, y);
      // y[n2 * P + k1] now holds the twiddled P-point results; Q-point DFTs over n2.
      gather_q<0>(x, y);
    }
  }

  // P-point DFTs over n1 for each n2, then twiddle by exp(S 2 pi i n2 k1 / R).
  template <int N2>
  static PSATD_HD __forceinline__ void split_stage(const cx<T>* x, cx<T>* y) {
    constexpr int P = smallest_factor<R>::v;
    constexpr int Q = R / P;
    if constexpr (N2 < Q) {
      cx<T> v[P];
#pragma unroll
      for (int n1 = 0; n1 < P; ++n1) v[n1] = x[Q * n1 + N2];
      dft<P, S, T>::run(v);
      twiddle_row<N2, 0>(v, y);
      split_stage<N2 + 1>(x, y);
    }
  }
  template <int N2, int K1>
  static PSATD_HD __forceinline__ void twiddle_row(const cx<T>* v, cx<T>* y) {
    constexpr int P = smallest_factor<R>::v;
    if constexpr (K1 < P) {
      y[N2 * P + K1] = twiddle_const<S, N2 * K1, R>(v[K1]);
      twiddle_row<N2, K1 + 1>(v, y);
    }
  }
  template <int K1>
  static PSATD_HD __forceinline__ void gather_q(cx<T>* x, const cx<T>* y) {
    constexpr int P = smallest_factor<R>::v;
    constexpr int Q = R / P;
    if constexpr (K1 < P) {
      cx<T> w[Q];
#pragma unroll
      for (int n2 = 0; n2 < Q; ++n2) w[n2] = y[n2 * P + K1];
      dft<Q, S, T>::run(w);
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) x[K1 + P * k2] = w[k2];
      gather_q<K1 + 1>(x, y);
    }
  }
};

}  // namespace psatd
