// Element-wise kernels of the two-step PML (Sec. 2.6): the full fields from their
// split parts, and the damped update of one set of split parts.
//
// Split parts, in array order: set A = E_xy, E_yz, E_zx, B_xy, B_yz, B_zx (component a
// driven by the derivative along axis a+1) and set B = E_xz, E_yx, E_zy, B_xz, B_yx,
// B_zy (along a+2).  The full component f (Ex Ey Ez Bx By Bz) is A[f] + B[f].  After the
// undamped advance, a part of set s (1 = A, 2 = B) of component a is multiplied by the
// damping factor exp(-sigma dt) of axis a+s at its cell.

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace psatd {
namespace {

constexpr int kPmlThreads = 256;

template <typename T>
struct Six {
  const T* in[6];
  T* out[6];
};

template <typename T>
__global__ void __launch_bounds__(kPmlThreads) k_pml_sum(Six<T> a, Six<T> b, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int f = 0; f < 6; ++f) a.out[f][i] = a.in[f][i] + b.in[f][i];
}

// parts[f] = (parts[f] + inc[f]) * damp_{axis(f)}[coordinate], box of NX x NY x NZ cells.
template <typename T>
__global__ void __launch_bounds__(kPmlThreads) k_pml_update(Six<T> io, const T* dx, const T* dy, const T* dz,
                                                              int set, int NX, int NY, int NZ) {
  const long long n = (long long)NX * NY * NZ;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % NX);
  const long long r = i / NX;
  const int y = (int)(r % NY), z = (int)(r / NY);
  const T d[3] = {dx[x], dy[y], dz[z]};
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int axis = (f % 3 + set) % 3;
    io.out[f][i] = (io.out[f][i] + io.in[f][i]) * d[axis];
  }
}

unsigned blocks(long long n) { return (unsigned)((n + kPmlThreads - 1) / kPmlThreads); }

}  // namespace

void launch_pml_sum(const void* const* parts, void* const* full, long long ncell, int fp64, hipStream_t s) {
  if (fp64) {
    Six<double> a{}, b{};
    for (int f = 0; f < 6; ++f) {
      a.in[f] = (const double*)parts[f];
      b.in[f] = (const double*)parts[6 + f];
      a.out[f] = (double*)full[f];
    }
    hipLaunchKernelGGL(k_pml_sum<double>, dim3(blocks(ncell)), dim3(kPmlThreads), 0, s, a, b, ncell);
  } else {
    Six<float> a{}, b{};
    for (int f = 0; f < 6; ++f) {
      a.in[f] = (const float*)parts[f];
      b.in[f] = (const float*)parts[6 + f];
      a.out[f] = (float*)full[f];
    }
    hipLaunchKernelGGL(k_pml_sum<float>, dim3(blocks(ncell)), dim3(kPmlThreads), 0, s, a, b, ncell);
  }
}

void launch_pml_update(void* const* parts, const void* const* inc, const void* const damp[3], int set, int NX,
                       int NY, int NZ, int fp64, hipStream_t s) {
  const long long n = (long long)NX * NY * NZ;
  if (fp64) {
    Six<double> io{};
    for (int f = 0; f < 6; ++f) {
      io.in[f] = (const double*)inc[f];
      io.out[f] = (double*)parts[f];
    }
    hipLaunchKernelGGL(k_pml_update<double>, dim3(blocks(n)), dim3(kPmlThreads), 0, s, io,
                       (const double*)damp[0], (const double*)damp[1], (const double*)damp[2], set, NX, NY, NZ);
  } else {
    Six<float> io{};
    for (int f = 0; f < 6; ++f) {
      io.in[f] = (const float*)inc[f];
      io.out[f] = (float*)parts[f];
    }
    hipLaunchKernelGGL(k_pml_update<float>, dim3(blocks(n)), dim3(kPmlThreads), 0, s, io,
                       (const float*)damp[0], (const float*)damp[1], (const float*)damp[2], set, NX, NY, NZ);
  }
}

}  // namespace psatd
