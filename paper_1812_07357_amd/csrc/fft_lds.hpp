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
#pragma once

#include "cplx.hpp"

namespace psatd {

constexpr int kMaxStages = 16;

struct LineSchedule {
  int n;
  int nstages;
  int radix[kMaxStages];
};

// Radices with a compiled stage; anything else must be factored by the host.
// (Keep in sync with the switch in lds_fft.)
inline constexpr int kRadices[] = {16, 13, 11, 9, 8, 7, 5, 4, 3, 2, 17};

template <typename T>
struct emax;  // register budget: complex values a thread holds through one stage
template <>
struct emax<float> { static constexpr int v = 32; };
template <>
struct emax<double> { static constexpr int v = 17; };

template <int R, int S, typename T>
__device__ __forceinline__ void stockham_stage(cx<T>* lds, int ld, int nlines, int n, int Ns,
                                               const Tw<T>* __restrict__ tw) {
  constexpr int MB = emax<T>::v / R;
  static_assert(MB >= 1, "radix larger than the register budget");
  const int bfl = n / R;
  const int total = nlines * bfl;
  const int nth = blockDim.x;
  const int tid = threadIdx.x;
  const int twstep = n / (Ns * R);
  cx<T> v[MB][R];
  int obase[MB];
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int j = tid + b * nth;
    obase[b] = -1;
    if (j < total) {
      const int line = j / bfl;
      const int jj = j - line * bfl;
      const int k = jj % Ns;
      const cx<T>* src = lds + line * ld + jj;
#pragma unroll
      for (int t = 0; t < R; ++t) v[b][t] = src[t * bfl];
      if (k != 0) {
#pragma unroll
        for (int t = 1; t < R; ++t) {
          v[b][t] = twmul<S>(v[b][t], tw[k * t * twstep]);
        }
      }
      dft<R, S, T>::run(v[b]);
      obase[b] = line * ld + (jj - k) * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    if (obase[b] >= 0) {
#pragma unroll
      for (int t = 0; t < R; ++t) lds[obase[b] + t * Ns] = v[b][t];
    }
  }
  __syncthreads();
}

// Full line transform of every line of the tile; S = -1 forward, +1 inverse
// (unnormalised).  `tw` holds w_n^m = exp(-2 pi i m / n), m in [0, n).
// Must be called by every thread of the block (it synchronises).
template <int S, typename T>
__device__ __forceinline__ void lds_fft(cx<T>* lds, int ld, int nlines, const LineSchedule& sch,
                                        const Tw<T>* __restrict__ tw) {
  int Ns = 1;
  const int n = sch.n;
  for (int s = 0; s < sch.nstages; ++s) {
    const int R = sch.radix[s];
    switch (R) {
      case 2: stockham_stage<2, S, T>(lds, ld, nlines, n, Ns, tw); break;
      case 3: stockham_stage<3, S, T>(lds, ld, nlines, n, Ns, tw); break;
      case 4: stockham_stage<4, S, T>(lds, ld, nlines, n, Ns, tw); break;
      case 5: stockham_stage<5, S, T>(lds, ld, nlines, n, Ns, tw); break;
      case 7: stockham_stage<7, S, T>(lds, ld, nlines, n, Ns, tw); break;
      case 8: stockham_stage<8, S, T>(lds, ld, nlines, n, Ns, tw); break;
      case 9: stockham_stage<9, S, T>(lds, ld, nlines, n, Ns, tw); break;
      case 11: stockham_stage<11, S, T>(lds, ld, nlines, n, Ns, tw); break;
      case 13: stockham_stage<13, S, T>(lds, ld, nlines, n, Ns, tw); break;
      case 16: stockham_stage<16, S, T>(lds, ld, nlines, n, Ns, tw); break;
      case 17: stockham_stage<17, S, T>(lds, ld, nlines, n, Ns, tw); break;
      default: break;  // the host never schedules another radix
    }
    Ns *= R;
  }
}

}  // namespace psatd
