// Plan-time tables, computed on the device in FP64 and stored at working precision.
//
// * FFT twiddles w_n^m = exp(-2 pi i m / n) (FP32: as hi + lo pairs of floats).
// * Order-p modified wavenumbers (Sec. 1.1 and 1.3 of arXiv:1812.07357: a
//   solver of order p uses a centred stencil of half width p/2; p = infinity is
//   the spectral derivative).  For the centred order-p first derivative on a
//   collocated grid the symbol is
//       k_p = sum_{l=1..m} b_l 2 sin(l k d) / d,  m = p / 2,
//   with b_1 = m / (m + 1) and b_{l+1} = -b_l l (m - l) / ((l + 1)(m + l + 1)).
//   The sine argument l k d = 2 pi l |m'| / n is reduced exactly in integers.
//   k_p is odd in k and zero at the Nyquist index (it is zero there for every
//   finite p, and kept zero at infinite order so that real fields stay real).
//   The staggered (Yee) variant uses the staggered difference instead (below).
// * PSATD coefficients per half-spectrum point, omega = c |K|, theta = omega dt:
//       C = cos theta, S1 = sin theta / omega, X1 = (1 - C) / omega^2,
//       X2 = (1 - S1/dt) / omega^2, X3 = (C - S1/dt) / omega^2,
//   from their Taylor series in theta^2 below theta = 0.1 (the direct forms
//   cancel catastrophically there), all multiplied by 1/(NX NY NZ) so that the
//   inverse transforms can stay unnormalised.

#include "internal.hpp"

namespace psatd {

namespace {

constexpr int kT = 256;

// FP32 twiddles are stored as hi + lo float pairs (hi = rounded value, lo = rounded remainder).
// Stores an FP64 complex value as a run-time twiddle of the working precision.
__device__ inline void put_tw(Tw<float>* dst, int i, double c, double s) {
  const float ch = (float)c, sh = (float)s;
  dst[i] = {{ch, sh}, {(float)(c - (double)ch), (float)(s - (double)sh)}};
}
__device__ inline void put_tw(Tw<double>* dst, int i, double c, double s) { dst[i] = {{c, s}}; }

// Stage-major twiddle table of a line schedule: entry (Ns - 1) + k (R - 1) + (t - 1)
// of the stage with radix R and span Ns is w_n^m, m = t k n / (Ns R) < n,
// evaluated in FP64 from the exact integer m.
struct StagePlan {
  int n, nstages;
  int radix[kMaxStages];
};

template <typename T>
__global__ void k_twiddles(Tw<T>* dst, StagePlan sp) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= sp.n - 1) return;
  int Ns = 1;
  for (int s = 0; s < sp.nstages; ++s) {
    const int R = sp.radix[s];
    if (e + 1 < Ns * R) {
      const int local = e + 1 - Ns;
      const int k = local / (R - 1), t = local - k * (R - 1) + 1;
      const long long m = (long long)t * k * (sp.n / (Ns * R));
      double sn, cs;
      sincospi(-2.0 * (double)m / (double)sp.n, &sn, &cs);
      put_tw(dst, e, cs, sn);
      return;
    }
    Ns *= R;
  }
}


// Bluestein chirp c[j] = exp(-i pi j^2 / n); j^2 is reduced modulo 2n exactly.
template <typename T>
__global__ void k_chirp(Tw<T>* dst, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const long long q = ((long long)j * j) % (2LL * n);
  double s, c;
  sincospi(-(double)q / (double)n, &s, &c);
  put_tw(dst, j, c, s);
}

// Bluestein filter F[k] = (1/m) sum_j b[j] exp(-2 pi i j k / m) with b[j] = b[m-j] = conj c[j]
// for 0 <= j < n and b = 0 elsewhere; direct FP64 sum (m is at most a few hundred).
template <typename T>
__global__ void k_bluestein_filter(Tw<T>* dst, int n, int m) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  double re = 0.0, im = 0.0;
  for (int j = 0; j < n; ++j) {
    const long long q = ((long long)j * j) % (2LL * n);
    double bs, bc;
    sincospi((double)q / (double)n, &bs, &bc);  // b[j] = exp(+i pi j^2 / n)
    const long long e = ((long long)j * k) % m;
    double es, ec;
    sincospi(2.0 * (double)e / (double)m, &es, &ec);
    // b[j] e^{-2 pi i j k / m}, and for j >= 1 the mirrored tap b[m-j] e^{+2 pi i j k / m}
    re += bc * ec + bs * es;
    im += bs * ec - bc * es;
    if (j >= 1 && 2 * j != m) {
      re += bc * ec - bs * es;
      im += bs * ec + bc * es;
    }
  }
  put_tw(dst, k, re / m, im / m);
}

// Staggered variant (Yee grid): the symbol of the order-p staggered difference,
//   k_s = sum_{l=1..m} a_l 2 sin((2l - 1) k d / 2) / d,
//   a_l = 1/(2l-1) prod_{j != l} (2j-1)^2 / ((2j-1)^2 - (2l-1)^2),
// or k itself at infinite order.  It does not vanish at the Nyquist index, which
// is taken at k = +pi/d (together with the half-cell shifts below).
__device__ double staggered_weight(int l, int m) {
  double a = 1.0 / (double)(2 * l - 1);
  const double ql = (double)(2 * l - 1) * (double)(2 * l - 1);
  for (int j = 1; j <= m; ++j)
    if (j != l) {
      const double qj = (double)(2 * j - 1) * (double)(2 * j - 1);
      a *= qj / (qj - ql);
    }
  return a;
}

__global__ void k_modk(double* dst, int n, int count, double d, int order, int staggered) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const long long ms = (2LL * i <= n) ? i : (long long)i - n;
  if (staggered) {
    const long long am = ms < 0 ? -ms : ms;
    double ks;
    if (order == 0) {
      ks = 2.0 * (double)am / ((double)n * d) * 3.14159265358979323846;
    } else {
      const int m = order / 2;
      double acc = 0.0;
      for (int l = 1; l <= m; ++l) {
        // sin((2l - 1) pi am / n), argument reduced modulo 2n exactly
        const long long num = ((2LL * l - 1) * am) % (2LL * n);
        acc += staggered_weight(l, m) * 2.0 * sinpi((double)num / (double)n);
      }
      ks = acc / d;
    }
    dst[i] = ms < 0 ? -ks : ks;
    return;
  }
  if (2LL * i == n) {  // Nyquist
    dst[i] = 0.0;
    return;
  }
  const long long am = ms < 0 ? -ms : ms;
  double kp;
  if (order == 0) {
    kp = 2.0 * (double)am / ((double)n * d) * 3.14159265358979323846;
  } else {
    const int m = order / 2;
    double b = (double)m / (double)(m + 1);
    double acc = 0.0;
    for (int l = 1; l <= m; ++l) {
      // sin(2 pi l am / n) with the argument reduced modulo n exactly
      const long long num = (2LL * l * am) % (2LL * n);
      acc += b * 2.0 * sinpi((double)num / (double)n);
      b = -b * (double)l * (double)(m - l) / ((double)(l + 1) * (double)(m + l + 1));
    }
    kp = acc / d;
  }
  dst[i] = ms < 0 ? -kp : kp;
}

// Staggered variant: kappa = k_s exp(i k d / 2) per DFT index (exact k; the
// Nyquist index at +pi/d), the symbol of the difference from a node to the half
// point above it; its conjugate goes from a half point down to the node.
template <typename T>
__global__ void k_shifted(const double* ks, cx<T>* dst, int n, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const long long ms = (2LL * i <= n) ? i : (long long)i - n;
  double sn, cs;
  sincospi((double)ms / (double)n, &sn, &cs);  // k d / 2 = pi ms / n
  dst[i] = {T(ks[i] * cs), T(ks[i] * sn)};
}

template <typename T>
__global__ void k_convert(const double* src, T* dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = T(src[i]);
}

template <typename T>
__global__ void k_coef(T* coef, const double* kx, const double* ky, const double* kz, int NXH, int NY, int NZ,
                       double dt, double c, double norm) {
  const long long npts = (long long)NXH * NY * NZ;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= npts) return;
  const int iz = (int)(q % NZ);
  const long long r = q / NZ;
  const int iy = (int)(r % NY);
  const int ix = (int)(r / NY);
  const double k2 = kx[ix] * kx[ix] + ky[iy] * ky[iy] + kz[iz] * kz[iz];
  const double om = c * sqrt(k2);
  const double th = om * dt;
  const double t2 = th * th;
  const double C = cos(th);
  double S1, X1, X2, X3;
  if (fabs(th) < 0.1) {
    const double dt2 = dt * dt;
    S1 = dt * (1.0 + t2 * (-1.0 / 6 + t2 * (1.0 / 120 + t2 * (-1.0 / 5040 + t2 * (1.0 / 362880)))));
    X1 = dt2 * (0.5 + t2 * (-1.0 / 24 + t2 * (1.0 / 720 + t2 * (-1.0 / 40320 + t2 * (1.0 / 3628800)))));
    X2 = dt2 * (1.0 / 6 + t2 * (-1.0 / 120 + t2 * (1.0 / 5040 + t2 * (-1.0 / 362880 + t2 * (1.0 / 39916800)))));
    X3 = dt2 * (-1.0 / 3 + t2 * (1.0 / 30 + t2 * (-1.0 / 840 + t2 * (1.0 / 45360 + t2 * (-1.0 / 3991680)))));
  } else {
    const double om2 = om * om;
    S1 = sin(th) / om;
    X1 = (1.0 - C) / om2;
    X2 = (1.0 - S1 / dt) / om2;
    X3 = (C - S1 / dt) / om2;
  }
  coef[q] = T(C * norm);
  coef[npts + q] = T(S1 * norm);
  coef[2 * npts + q] = T(X1 * norm);
  coef[3 * npts + q] = T(X2 * norm);
  coef[4 * npts + q] = T(X3 * norm);
}

inline unsigned nblk(long long n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace

void launch_twiddles(void* dst, const LineSchedule& sch, int fp64, hipStream_t s) {
  StagePlan sp{sch.n, sch.nstages, {}};
  for (int i = 0; i < sch.nstages; ++i) sp.radix[i] = sch.radix[i];
  if (sch.n < 2) return;
  if (fp64)
    hipLaunchKernelGGL(k_twiddles<double>, dim3(nblk(sch.n)), dim3(kT), 0, s, (Tw<double>*)dst, sp);
  else
    hipLaunchKernelGGL(k_twiddles<float>, dim3(nblk(sch.n)), dim3(kT), 0, s, (Tw<float>*)dst, sp);
}

void launch_bluestein(void* chirp, void* filt, int n, int m, int fp64, hipStream_t s) {
  if (fp64) {
    hipLaunchKernelGGL(k_chirp<double>, dim3(nblk(n)), dim3(kT), 0, s, (Tw<double>*)chirp, n);
    hipLaunchKernelGGL(k_bluestein_filter<double>, dim3(nblk(m)), dim3(kT), 0, s, (Tw<double>*)filt, n, m);
  } else {
    hipLaunchKernelGGL(k_chirp<float>, dim3(nblk(n)), dim3(kT), 0, s, (Tw<float>*)chirp, n);
    hipLaunchKernelGGL(k_bluestein_filter<float>, dim3(nblk(m)), dim3(kT), 0, s, (Tw<float>*)filt, n, m);
  }
}

void launch_modk(double* dst, int n, int count, double d, int order, int staggered, hipStream_t s) {
  hipLaunchKernelGGL(k_modk, dim3(nblk(count)), dim3(kT), 0, s, dst, n, count, d, order, staggered);
}

void launch_shifted(const double* ks, void* dst, int n, int count, int fp64, hipStream_t s) {
  if (fp64)
    hipLaunchKernelGGL(k_shifted<double>, dim3(nblk(count)), dim3(kT), 0, s, ks, (cx<double>*)dst, n, count);
  else
    hipLaunchKernelGGL(k_shifted<float>, dim3(nblk(count)), dim3(kT), 0, s, ks, (cx<float>*)dst, n, count);
}

void launch_coef(void* coef, void* kxw, void* kyw, void* kzw, const double* kx, const double* ky,
                 const double* kz, int NXH, int NY, int NZ, double dt, double c, double norm, int fp64,
                 hipStream_t s) {
  const long long npts = (long long)NXH * NY * NZ;
  if (fp64) {
    hipLaunchKernelGGL(k_coef<double>, dim3(nblk(npts)), dim3(kT), 0, s, (double*)coef, kx, ky, kz, NXH, NY, NZ,
                       dt, c, norm);
    hipLaunchKernelGGL(k_convert<double>, dim3(nblk(NXH)), dim3(kT), 0, s, kx, (double*)kxw, NXH);
    hipLaunchKernelGGL(k_convert<double>, dim3(nblk(NY)), dim3(kT), 0, s, ky, (double*)kyw, NY);
    hipLaunchKernelGGL(k_convert<double>, dim3(nblk(NZ)), dim3(kT), 0, s, kz, (double*)kzw, NZ);
  } else {
    hipLaunchKernelGGL(k_coef<float>, dim3(nblk(npts)), dim3(kT), 0, s, (float*)coef, kx, ky, kz, NXH, NY, NZ,
                       dt, c, norm);
    hipLaunchKernelGGL(k_convert<float>, dim3(nblk(NXH)), dim3(kT), 0, s, kx, (float*)kxw, NXH);
    hipLaunchKernelGGL(k_convert<float>, dim3(nblk(NY)), dim3(kT), 0, s, ky, (float*)kyw, NY);
    hipLaunchKernelGGL(k_convert<float>, dim3(nblk(NZ)), dim3(kT), 0, s, kz, (float*)kzw, NZ);
  }
}

}  // namespace psatd
