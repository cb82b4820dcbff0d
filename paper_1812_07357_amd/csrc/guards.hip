// Standalone guard fill / merge between the periodic global grid G1 and box arrays.
//
// Sec. 2.5.2 of arXiv:1812.07357: (1) G1 is copied into G2 including the
// guard cells, which are filled from G1 itself (here: the periodic wrap of the
// global index); (3) after the solve the interior, without guards, is copied
// back from G2 to G1.  The add mode sums every box cell (guards included)
// into its wrapped global cell, for sources deposited on boxes; a thread owns
// one global cell and sums its pre-images in a fixed order (no atomics).

#include "internal.hpp"

namespace psatd {

namespace {

constexpr int kT = 256;
constexpr int kMaxFields = 16;

struct PtrSet {
  const void* in[kMaxFields];
  void* out[kMaxFields];
};

template <typename T>
__global__ void k_fill(PtrSet ps, int BX, int BY, int BZ, int sx, int sy, int sz, int GX, int GY, int GZ) {
  const long long nbox = (long long)BX * BY * BZ;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nbox) return;
  const int f = blockIdx.y;
  const int i = (int)(q % BX);
  const long long r = q / BX;
  const int j = (int)(r % BY);
  const int k = (int)(r / BY);
  const long long xg = ((long long)sx + i) % GX;
  const long long yg = ((long long)sy + j) % GY;
  const long long zg = ((long long)sz + k) % GZ;
  const T* src = (const T*)ps.in[f];
  T* dst = (T*)ps.out[f];
  dst[q] = src[(zg * GY + yg) * GX + xg];
}

template <typename T>
__global__ void k_merge_copy(PtrSet ps, int BX, int BY, int gx, int gy, int gz, int nx, int ny, int nz, int ox,
                             int oy, int oz, int GX, int GY, int GZ) {
  const long long nint = (long long)nx * ny * nz;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nint) return;
  const int f = blockIdx.y;
  const int i = (int)(q % nx);
  const long long r = q / nx;
  const int j = (int)(r % ny);
  const int k = (int)(r / ny);
  const T* src = (const T*)ps.in[f];
  T* dst = (T*)ps.out[f];
  const long long xg = ((long long)ox + i) % GX;
  const long long yg = ((long long)oy + j) % GY;
  const long long zg = ((long long)oz + k) % GZ;
  dst[(zg * GY + yg) * GX + xg] = src[((long long)(k + gz) * BY + (j + gy)) * BX + (i + gx)];
}

// One thread per global cell covered by the box; pre-images along an axis are a, a+G, a+2G, ... < B.
template <typename T>
__global__ void k_merge_add(PtrSet ps, int BX, int BY, int BZ, int sx, int sy, int sz, int GX, int GY, int GZ) {
  const int cx = BX < GX ? BX : GX;
  const int cy = BY < GY ? BY : GY;
  const int cz = BZ < GZ ? BZ : GZ;
  const long long ncov = (long long)cx * cy * cz;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ncov) return;
  const int f = blockIdx.y;
  const int a = (int)(q % cx);
  const long long r = q / cx;
  const int b = (int)(r % cy);
  const int c = (int)(r / cy);
  const T* src = (const T*)ps.in[f];
  T* dst = (T*)ps.out[f];
  T acc = T(0);
  for (int k = c; k < BZ; k += GZ)
    for (int j = b; j < BY; j += GY)
      for (int i = a; i < BX; i += GX) acc += src[((long long)k * BY + j) * BX + i];
  const long long xg = ((long long)sx + a) % GX;
  const long long yg = ((long long)sy + b) % GY;
  const long long zg = ((long long)sz + c) % GZ;
  dst[(zg * GY + yg) * GX + xg] += acc;
}

inline unsigned nblk(long long n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace

void launch_guard_fill(const void* const* g1, void* const* box, int nfields, int esize, const int bd[3],
                       const int start[3], const int gd[3], hipStream_t s) {
  PtrSet ps{};
  for (int f = 0; f < nfields; ++f) {
    ps.in[f] = g1[f];
    ps.out[f] = box[f];
  }
  const long long n = (long long)bd[0] * bd[1] * bd[2];
  dim3 grid(nblk(n), (unsigned)nfields);
  if (esize == 8)
    hipLaunchKernelGGL(k_fill<double>, grid, dim3(kT), 0, s, ps, bd[0], bd[1], bd[2], start[0], start[1], start[2],
                       gd[0], gd[1], gd[2]);
  else
    hipLaunchKernelGGL(k_fill<float>, grid, dim3(kT), 0, s, ps, bd[0], bd[1], bd[2], start[0], start[1], start[2],
                       gd[0], gd[1], gd[2]);
}

void launch_guard_merge(const void* const* box, void* const* g1, int nfields, int esize, const int bd[3],
                        const int guard[3], const int interior[3], const int origin[3], const int gd[3], int mode,
                        hipStream_t s) {
  PtrSet ps{};
  for (int f = 0; f < nfields; ++f) {
    ps.in[f] = box[f];
    ps.out[f] = g1[f];
  }
  if (mode == 0) {
    const long long n = (long long)interior[0] * interior[1] * interior[2];
    dim3 grid(nblk(n), (unsigned)nfields);
    if (esize == 8)
      hipLaunchKernelGGL(k_merge_copy<double>, grid, dim3(kT), 0, s, ps, bd[0], bd[1], guard[0], guard[1], guard[2],
                         interior[0], interior[1], interior[2], origin[0], origin[1], origin[2], gd[0], gd[1], gd[2]);
    else
      hipLaunchKernelGGL(k_merge_copy<float>, grid, dim3(kT), 0, s, ps, bd[0], bd[1], guard[0], guard[1], guard[2],
                         interior[0], interior[1], interior[2], origin[0], origin[1], origin[2], gd[0], gd[1], gd[2]);
  } else {
    int start[3];
    for (int a = 0; a < 3; ++a) start[a] = (int)((((long long)origin[a] - guard[a]) % gd[a] + gd[a]) % gd[a]);
    const long long n = (long long)(bd[0] < gd[0] ? bd[0] : gd[0]) * (bd[1] < gd[1] ? bd[1] : gd[1]) *
                        (bd[2] < gd[2] ? bd[2] : gd[2]);
    dim3 grid(nblk(n), (unsigned)nfields);
    if (esize == 8)
      hipLaunchKernelGGL(k_merge_add<double>, grid, dim3(kT), 0, s, ps, bd[0], bd[1], bd[2], start[0], start[1],
                         start[2], gd[0], gd[1], gd[2]);
    else
      hipLaunchKernelGGL(k_merge_add<float>, grid, dim3(kT), 0, s, ps, bd[0], bd[1], bd[2], start[0], start[1],
                         start[2], gd[0], gd[1], gd[2]);
  }
}

}  // namespace psatd
