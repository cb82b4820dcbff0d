// Internal interface between the host runtime (plan.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_lds.hpp"

namespace psatd {

using i64 = long long;

// Intermediate layouts of the half spectrum (box of NX x NY x NZ cells, NXH = NX/2 + 1):
//   layout A  [field][z][kx][y]   (y fastest)  -- after the x pass
//   layout B  [field][kx][ky][z]  (z fastest)  -- after the y pass, k-space push in place
// Every pass reads whole contiguous lines on one side and writes tiles of
// consecutive lines (a short contiguous run per position) on the other.

// P1: x-axis real-to-complex transform of pairs of y-lines (two real lines form
// one complex line), box arrays or a periodic gather from G1, into layout A.
template <typename T>
struct XFwdParams {
  const T* src[11];
  cx<T>* dst;            // layout A, nfields * NZ * NXH * NY
  i64 src_extent;        // elements in each source array
  i64 dst_extent;        // elements in dst
  int NX, NY, NZ, NXH;
  int ty;                // real y-lines per tile (even)
  int ytiles;
  int gather;            // 0: src is box shaped; 1: src is G1 (GX, GY, GZ) with wrap
  int GX, GY, GZ;
  int x0, y0, z0;        // (origin - nguard) mod G, non-negative
  LineSchedule sch;
  const Tw<T>* tw;
};

// P2 / P4: transform along the middle index of a tile of lines and transpose.
// A line u of field f at outer index o is at  base_in + f*fs_in + o*os_in + u*ls_in + p*ps_in.
template <typename T>
struct YPassParams {
  const cx<T>* in;
  cx<T>* out;
  i64 in_extent, out_extent;
  i64 fs_in, os_in, ls_in, ps_in;
  i64 fs_out, os_out, ls_out, ps_out;
  int n;                 // line length
  int nl;                // lines per tile
  int u_lo, u_hi;        // lines processed: [u_lo, u_hi)
  int utiles;            // tiles along u
  int p_lo, p_hi;        // output positions written: [p_lo, p_hi)
  LineSchedule sch;
  const Tw<T>* tw;
};

// P3: z-axis forward transform of 11 fields, k-space push, inverse z transform of E, B.
template <typename T>
struct ZPushParams {
  cx<T>* b;              // layout B, 11 fields of npts each
  i64 npts;              // NXH * NY * NZ
  const T* coef;         // C, S1, X1, X2, X3 each npts, pre-scaled by 1/(NX NY NZ)
  const T* kx;           // NXH
  const T* ky;           // NY
  const T* kz;           // NZ
  int NY, NZ, NXH;
  int z_lo, z_hi;        // output z written: [z_lo, z_hi)
  T c2;                  // c^2
  T inv_eps0;            // 1 / eps0
  LineSchedule sch;
  const Tw<T>* tw;
};

// P5: x-axis complex-to-real inverse of pairs of y-lines from layout A, to box
// arrays or scattered into the interior of G1.
template <typename T>
struct XInvParams {
  const cx<T>* src;      // layout A
  T* dst[6];
  i64 src_extent;
  i64 dst_extent;        // elements in each destination array
  int NX, NY, NZ, NXH;
  int ty;                // real y-lines per tile (even)
  int y_lo, y_hi;        // y-lines processed
  int z_lo, z_hi;        // z-planes processed
  int ytiles;
  int scatter;           // 0: dst is box shaped; 1: dst is G1, interior only
  int GX, GY, GZ;
  int ox, oy, oz;        // origin of the interior in G1
  int gx, gy, gz;        // guard widths
  int nx;                // interior cells along x
  LineSchedule sch;
  const Tw<T>* tw;
};

template <typename T>
void launch_xfwd(const XFwdParams<T>& p, int nfields, int nthreads, hipStream_t s);
template <typename T>
void launch_ypass(const YPassParams<T>& p, int nfields, int nouter, int inverse, int nthreads, hipStream_t s);
template <typename T>
void launch_zpush(const ZPushParams<T>& p, int nthreads, hipStream_t s);
template <typename T>
void launch_xinv(const XInvParams<T>& p, int nfields, int nthreads, hipStream_t s);

// Tables (FP64 math, stored at working precision).
void launch_twiddles(void* dst, int n, int fp64, hipStream_t s);
void launch_modk(double* dst, int n, int count, double d, int order, hipStream_t s);
void launch_coef(void* coef, void* kxw, void* kyw, void* kzw, const double* kx, const double* ky,
                 const double* kz, int NXH, int NY, int NZ, double dt, double c, double norm, int fp64,
                 hipStream_t s);

// Standalone guard fill / merge (element-wise gathers).
void launch_guard_fill(const void* const* g1, void* const* box, int nfields, int esize, const int box_dims[3],
                       const int start[3], const int gdims[3], hipStream_t s);
void launch_guard_merge(const void* const* box, void* const* g1, int nfields, int esize, const int box_dims[3],
                        const int guard[3], const int interior[3], const int origin[3], const int gdims[3],
                        int mode, hipStream_t s);

}  // namespace psatd
