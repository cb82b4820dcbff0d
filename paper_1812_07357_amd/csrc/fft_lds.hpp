// Line FFTs on tiles held in LDS: mixed-radix Stockham (self-sorting) stages.
//
// A tile holds `nlines` lines of length n, line l starting at lds + l * ld.
// Stage s with radix R and span Ns (product of the earlier radices) treats
// butterfly j in [0, n/R) of each line as
//   v[t] = x[j + t n/R]                      (t = 0..R-1)
//   v[t] *= w_n^(S * t * k * n/(Ns R)),       k = j mod Ns
//   V = DFT_R(v)
//   y[(j - k) R + k + t Ns] = V[t]
// which leaves the transform in natural order after the last stage.  The
// stage runs in place: every thread first reads all of its butterflies into
// registers, the block synchronises, then every thread writes.
//
// Twiddle table layout (stage-major): the R-1 twiddles of butterfly k of the
// stage with span Ns are consecutive, at tw[(Ns - 1) + k (R - 1) + (t - 1)]
// = w_n^(t k n/(Ns R)) for t = 1..R-1.  The stages' blocks telescope to
// n - 1 entries in all, and a butterfly reads its twiddles from one base
// address at fixed offsets.
//
// Element i of a line lives at LDS slot i + i/16 of that line: the first stage
// writes with a stride of R elements, and without the padding slot every
// lane of a 16-lane group would hit the same LDS bank for R = 16.
#pragma once

#include "cplx.hpp"

#include <cstdint>

namespace psatd {

constexpr int kMaxStages = 16;

// Division by a run-time constant d via a multiply-high: q = (mulhi(x, m) + x) >> s,
// exact for 0 <= x < 2^31 (s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1).
struct FastDiv {
  uint32_t d, m, s;
};
inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f{d, 0, 0};
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  f.s = s;
  f.m = (uint32_t)((((1ull << 32) * ((1ull << s) - d)) / d) + 1);
  return f;
}
__device__ __forceinline__ int fdiv(int x, const FastDiv& f) {
  return (int)((__umulhi((uint32_t)x, f.m) + (uint32_t)x) >> f.s);
}

struct LineSchedule {
  int n;
  int nstages;
  int radix[kMaxStages];
  FastDiv bfl[kMaxStages];  // n / radix[s]
  FastDiv ns[kMaxStages];   // product of radix[0..s-1]
};

template <typename T>
struct emax;  // register budget: complex values a thread holds through one stage
template <>
struct emax<float> { static constexpr int v = 17; };
template <>
struct emax<double> { static constexpr int v = 17; };

// i + floor(i / 16) == floor(17 i / 16) for 0 <= i < 2^27: one multiply-shift, and a
// sequence i0 + t d becomes a running sum of 17 d.
__host__ __device__ __forceinline__ int lpad(int i) { return (int)((17u * (uint32_t)i) >> 4); }
// floor(q / 16): with q = 17 i + 16 base this is base + lpad(i).
__device__ __forceinline__ int pad_slot(uint32_t q) { return (int)(q >> 4); }
// LDS slots per line of n elements (odd, so that lanes walking across lines use distinct banks).
__host__ __device__ __forceinline__ int lds_line(int n) { return (lpad(n - 1) + 1) | 1; }

template <int R, int S, typename T>
__device__ __forceinline__ void stockham_stage(cx<T>* lds, int ld, int nlines, int n, int Ns, const FastDiv& fb,
                                               const FastDiv& fn, const Tw<T>* __restrict__ tw) {
  // butterflies per thread: as many as the register budget holds, at least one
  // (radices above the budget hold one butterfly of R values)
  constexpr int MB = emax<T>::v / R > 0 ? emax<T>::v / R : 1;
  const int bfl = (int)fb.d;
  const int total = nlines * bfl;
  const int nth = blockDim.x;
  const int tid = threadIdx.x;
  const uint32_t dq_in = 17u * (uint32_t)bfl, dq_out = 17u * (uint32_t)Ns;
  cx<T> v[MB][R];
  int lbase[MB];  // LDS offset of the butterfly's line, -1 if none
  int obase[MB];  // first output position (jj - k) R + k within the line
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int j = tid + b * nth;
    lbase[b] = -1;
    obase[b] = 0;
    if (j < total) {
      const int line = fdiv(j, fb);
      const int jj = j - line * bfl;
      const int k = jj - fdiv(jj, fn) * Ns;
      // slot of element jj + t bfl of the line: line * ld + floor(q / 16) with
      // q = 17 (jj + t bfl) kept as a running sum (the line offset folded in as 16 line * ld)
      uint32_t q = 17u * (uint32_t)jj + 16u * (uint32_t)(line * ld);
#pragma unroll
      for (int t = 0; t < R; ++t) {
        v[b][t] = lds[pad_slot(q)];
        q += dq_in;
      }
      if (Ns > 1) {  // uniform; the k = 0 entries are exactly 1
        const Tw<T>* w = tw + (Ns - 2) + k * (R - 1);
#pragma unroll
        for (int t = 1; t < R; ++t) v[b][t] = twmul<S>(v[b][t], w[t]);
      }
      dft<R, S, T>::run(v[b]);
      lbase[b] = line * ld;
      obase[b] = (jj - k) * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    if (lbase[b] >= 0) {
      uint32_t q = 17u * (uint32_t)obase[b] + 16u * (uint32_t)lbase[b];
#pragma unroll
      for (int t = 0; t < R; ++t) {
        lds[pad_slot(q)] = v[b][t];
        q += dq_out;
      }
    }
  }
  __syncthreads();
}

// Full line transform of every line of the tile; S = -1 forward, +1 inverse
// (unnormalised).  `tw` is the stage-major twiddle table of `sch` (forward
// sign, w_n = exp(-2 pi i / n); the inverse conjugates).
// Must be called by every thread of the block (it synchronises).
template <int S, typename T>
__device__ __forceinline__ void lds_fft(cx<T>* lds, int ld, int nlines, const LineSchedule& sch,
                                        const Tw<T>* __restrict__ tw) {
  int Ns = 1;
  const int n = sch.n;
  for (int s = 0; s < sch.nstages; ++s) {
    const int R = sch.radix[s];
    const FastDiv& fb = sch.bfl[s];
    const FastDiv& fn = sch.ns[s];
    switch (R) {
      case 2: stockham_stage<2, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 3: stockham_stage<3, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 4: stockham_stage<4, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 5: stockham_stage<5, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 7: stockham_stage<7, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 8: stockham_stage<8, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 9: stockham_stage<9, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 11: stockham_stage<11, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 13: stockham_stage<13, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 6: stockham_stage<6, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 10: stockham_stage<10, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 12: stockham_stage<12, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 16: stockham_stage<16, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 17: stockham_stage<17, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 18: stockham_stage<18, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 20: stockham_stage<20, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 24: stockham_stage<24, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 32: stockham_stage<32, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      case 36: stockham_stage<36, S, T>(lds, ld, nlines, n, Ns, fb, fn, tw); break;
      default: break;  // the host never schedules another radix
    }
    Ns *= R;
  }
}

// One line transform as the passes see it: either direct (the stages of
// `sch` run over the line length n) or Bluestein's chirp-z form for lengths with
// a prime factor that has no compiled radix.  With c[j] = exp(-i pi j^2 / n),
//   X[k] = c[k] sum_j (x[j] c[j]) conj(c[k - j]),
// a linear convolution evaluated as a cyclic one of padded length m >= 2n - 1:
// premultiply by c, transform (length m), multiply by the transform of the
// chirp filter b (b[j] = b[m-j] = conj c[j] for 0 <= j < n, zero elsewhere,
// scaled by 1/m), inverse transform, postmultiply by c.  The inverse DFT uses
// the conjugate chirp and filter (b is even, so its transform is too).
template <typename T>
struct LineFFT {
  LineSchedule sch;     // stages over the transform length (n, or m for Bluestein)
  const Tw<T>* tw;      // twiddles of that length
  int n;                // line length
  int blue;             // 1: Bluestein, padded length sch.n
  FastDiv fd_n, fd_m;   // n and sch.n
  const Tw<T>* chirp;   // n entries c[j]
  const Tw<T>* filt;    // sch.n entries: transform of b, over m
};

// LDS slots needed per line by a LineFFT.
__host__ __device__ __forceinline__ int fft_slots(int transform_len) { return lds_line(transform_len); }

template <int S, typename T>
__device__ __forceinline__ void lds_line_fft(cx<T>* lds, int ld, int nlines, const LineFFT<T>& L) {
  if (!L.blue) {
    lds_fft<S, T>(lds, ld, nlines, L.sch, L.tw);
    return;
  }
  const int n = L.n, m = L.sch.n;
  const int nth = blockDim.x;
  for (int e = threadIdx.x; e < nlines * m; e += nth) {
    const int line = fdiv(e, L.fd_m);
    const int j = e - line * m;
    cx<T>* s = lds + line * ld + lpad(j);
    *s = (j < n) ? twmul<S>(*s, L.chirp[j]) : cx<T>{T(0), T(0)};
  }
  __syncthreads();
  lds_fft<-1, T>(lds, ld, nlines, L.sch, L.tw);
  for (int e = threadIdx.x; e < nlines * m; e += nth) {
    const int line = fdiv(e, L.fd_m);
    const int j = e - line * m;
    cx<T>* s = lds + line * ld + lpad(j);
    *s = twmul<S>(*s, L.filt[j]);
  }
  __syncthreads();
  lds_fft<1, T>(lds, ld, nlines, L.sch, L.tw);
  for (int e = threadIdx.x; e < nlines * n; e += nth) {
    const int line = fdiv(e, L.fd_n);
    const int j = e - line * n;
    cx<T>* s = lds + line * ld + lpad(j);
    *s = twmul<S>(*s, L.chirp[j]);
  }
  __syncthreads();
}

}  // namespace psatd
