// Internal interface between the host runtime (plan.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_lds.hpp"
#include "gmem.hpp"

namespace psatd {

using i64 = long long;

// Intermediate layouts of the half spectrum (box of NX x NY x NZ cells, NXH = NX/2 + 1):
//   layout A  [field][z][kx][y]   (y fastest)  -- after the x pass
//   layout B  [field][kx][ky][z]  (z fastest)  -- after the y pass, k-space push in place
// Every pass reads whole contiguous lines on one side and writes tiles of
// consecutive lines (a short contiguous run per position) on the other.

// Every pass runs as a persistent kernel: a grid sized to the resident capacity
// walks over the pass's tiles; several blocks share a CU and overlap one
// another's loads, transforms and barriers.  Arrays are addressed through
// buffer resources (see gmem.hpp), one resource per field.

// P1: x-axis real-to-complex transform of pairs of y-lines (two real lines form
// one complex line), box arrays or a periodic gather from G1, into layout A.
template <typename T>
struct XFwdParams {
  const T* src[11];
  uint32_t src_bytes;    // bytes of each source array
  cx<T>* dst;            // layout A; field f starts at dst + f * npts
  i64 npts;
  uint32_t dst_bytes;    // bytes of one field of A
  int NX, NY, NZ, NXH;
  int ty;                // real y-lines per tile (even)
  int ytiles, ntiles;    // tiles per (field, z) and in total
  int gather;            // 0: src is box shaped; 1: src is G1 (GX, GY, GZ) with wrap
  int xtab;              // gather through a per-tile LDS table (wrapped x of every column,
                         // G1 offset of every real row) placed after the tile's lines
  int GX, GY, GZ;
  int x0, y0, z0;        // (origin - nguard) mod G, non-negative
  FastDiv fd_ytiles, fd_NZ, fd_NX, fd_GX, fd_GY, fd_GZ, fd_nc;
  int ld_drow, ld_dcol;  // block stride over (complex line, x) = divmod(threads, NX)
  int wr_drow, wr_dcol;  // block stride over (kx, complex line) = divmod(threads, ty / 2)
  int ra, rb;            // two-stage kernel with compile-time radices (ty = 2 kXTwoStageLines), or 0, 0
  LineFFT<T> fft;
};

// P2 / P4: transform along the middle index of a tile of lines and transpose.
// Element p of line u of field f at outer index o is at
//   in + f*fs_in + o*os_in + u*ls_in + p*ps_in   (elements).
template <typename T>
struct YPassParams {
  const cx<T>* in;
  cx<T>* out;
  i64 fs_in, fs_out;
  uint32_t in_bytes, out_bytes;  // bytes of one field
  int os_in, ls_in, ps_in;
  int os_out, ls_out, ps_out;
  int n;                 // line length
  int nl, nl_last;       // lines per tile (last tile: nl_last)
  int u_lo, u_hi;        // lines processed: [u_lo, u_hi)
  int utiles, nouter, ntiles;
  int p_lo, p_hi;        // output positions written: [p_lo, p_hi)
  int ra, rb;            // two-stage kernel with compile-time radices (ra, rb) and
                         // kYTwoStageLines lines per tile, or 0, 0
  FastDiv fd_utiles, fd_nouter, fd_n, fd_nl, fd_nl_last, fd_np;
  LineFFT<T> fft;
};

// P3: z-axis forward transform of 11 fields, k-space push, inverse z transform of E, B.
template <typename T>
struct ZPushParams {
  cx<T>* b;              // layout B, 11 fields of npts each
  i64 npts;              // NXH * NY * NZ
  uint32_t field_bytes;  // bytes of one field
  const T* coef;         // C, S1, X1, X2, X3 each npts, pre-scaled by 1/(NX NY NZ)
  uint32_t coef_bytes;   // bytes of one table
  const T* kx;           // NXH
  const T* ky;           // NY
  const T* kz;           // NZ
  // Staggered grid (stag = 1): kappa = k_s exp(i k d / 2) per index, the symbol of
  // a difference from the nodes to the half points above them (its conjugate for
  // the way back); kx, ky, kz then hold k_s.
  int stag;
  const cx<T>* kxc;      // NXH
  const cx<T>* kyc;      // NY
  const cx<T>* kzc;      // NZ
  int NY, NZ, NXH;
  int ncol;              // (kx, ky) columns per tile
  int zgroup;            // lines per transform call (the lines of a tile are transformed in groups)
  int ntiles;            // ceil(NXH * NY / ncol)
  int z_lo, z_hi;        // output z written: [z_lo, z_hi)
  int ra, rb;            // two-stage kernel with compile-time radices (ra, rb), or 0, 0
  T c2;                  // c^2
  T inv_eps0;            // 1 / eps0
  // Two-step PML (split fields): 0 = ordinary push; 1 = write the increments of the
  // twelve split parts over the step (set A to fields 0..5, set B to 6..11 of b, which
  // then holds 12 fields); dt and 1/(NX NY NZ) for the terms without a table.
  int pml;
  T dt, inv_n;
  FastDiv fd_NY, fd_NZ, fd_ncol;
  LineFFT<T> fft;
};

// P5: x-axis complex-to-real inverse of pairs of y-lines from layout A, to box
// arrays or scattered into the interior of G1.
template <typename T>
struct XInvParams {
  const cx<T>* src;      // layout A
  i64 npts;
  uint32_t src_bytes;    // bytes of one field of A
  T* dst[6];
  uint32_t dst_bytes;    // bytes of each destination array
  int NX, NY, NZ, NXH;
  int ty;                // real y-lines per tile (even)
  int y_lo, y_hi;        // y-lines processed
  int z_lo, z_hi;        // z-planes processed
  int ytiles, ntiles;
  int scatter;           // 0: dst is box shaped; 1: dst is G1, interior only
  int GX, GY, GZ;
  int ox, oy, oz;        // origin of the interior in G1
  int gx, gy, gz;        // guard widths
  int nx;                // interior cells along x
  FastDiv fd_ytiles, fd_nz, fd_nc, fd_NX, fd_GX, fd_GY, fd_GZ;
  int nthreads;          // block size the tile was fitted for (kXInvThreads, or kLineThreads
                         // when a line's butterflies exceed the smaller block)
  int ra, rb;            // two-stage kernel with compile-time radices (ty = 2 kXTwoStageLines), or 0, 0
  LineFFT<T> fft;
};

// Line schedules (RA, RB), N = RA * RB, with a compiled two-stage z kernel
// (single-column tiles of 256 threads, every offset a compile-time constant).
constexpr int kZTwoStage[][2] = {{16, 20}, {20, 16}, {16, 16}, {24, 24}, {32, 17}, {17, 32}};
constexpr int kZTwoStageThreads = 256;
// LDS slots per line of the two-stage kernel: the intermediate rows of RB
// butterflies padded to RA | 1 slots, or the N points in natural order.
constexpr int two_stage_slots(int ra, int rb) { return ((rb * (ra | 1) > ra * rb) ? rb * (ra | 1) : ra * rb) | 1; }

// Line schedules (RA, RB) with compiled two-stage y kernels, their lines per tile,
// LDS slots per line (RB padded rows of RA | 1 slots) and block size (one
// butterfly per thread in either stage).
constexpr int kYTwoStage[][2] = {{16, 20}, {20, 16}, {16, 16}, {24, 24}, {32, 17}, {17, 32}};
constexpr int kYTwoStageLines = 16;
constexpr int two_stage_y_slots(int ra, int rb) { return (rb * (ra | 1)) | 1; }
constexpr int two_stage_y_threads(int ra, int rb) {
  return ((kYTwoStageLines * (ra > rb ? ra : rb) + 63) / 64) * 64;
}

// Line schedules (RA, RB) with compiled two-stage x kernels (single boxes), complex
// lines (pairs of real rows) per tile, and block size (one butterfly per thread).
constexpr int kXTwoStage[][2] = {{24, 24}, {32, 18}, {18, 32}, {16, 20}, {20, 16}, {16, 16}, {32, 17}, {17, 32}};
constexpr int kXTwoStageLines = 8;
constexpr int two_stage_x_threads(int ra, int rb) {
  return ((kXTwoStageLines * (ra > rb ? ra : rb) + 63) / 64) * 64;
}

// Threads per block of the x and y passes.
constexpr int kLineThreads = 512;
// Threads per block of the x inverse pass: its tiles hold the same lines as the
// x forward pass's (as far as the butterfly budget allows) in smaller blocks, so
// more of them share a CU; lines too long for it fall back to kLineThreads.
constexpr int kXInvThreads = 256;
// Block sizes of the z pass (tried in this order; the first whose line butterflies fit is used).
constexpr int kZThreads[2] = {256, 512};
// Complex values a thread loads from global memory before moving them to LDS
// (one round of a tile load; a tile takes as many rounds as it needs).
template <typename T>
struct load_round;
template <>
struct load_round<float> { static constexpr int v = 12; };
template <>
struct load_round<double> { static constexpr int v = 12; };

// A batch of boxes for one pass: per-box parameters in device memory; the tiles
// of box b are numbered starts[b] .. starts[b+1]-1 (starts[nbox] == total).
template <typename P>
struct BatchArgs {
  const P* descs;
  const int* starts;
  int nbox;
  int total;
};

template <typename T>
size_t xfwd_lds(const XFwdParams<T>& p);
template <typename T>
size_t ypass_lds(const YPassParams<T>& p);
template <typename T>
size_t zpush_lds(const ZPushParams<T>& p);
template <typename T>
size_t xinv_lds(const XInvParams<T>& p);

template <typename T>
void launch_xfwd_batch(const BatchArgs<XFwdParams<T>>& a, size_t lds, hipStream_t s);
template <typename T>
void launch_ypass_batch(const BatchArgs<YPassParams<T>>& a, int inverse, size_t lds, hipStream_t s);
template <typename T>
void launch_zpush_batch(const BatchArgs<ZPushParams<T>>& a, int nthreads, size_t lds, hipStream_t s);
template <typename T>
void launch_xinv_batch(const BatchArgs<XInvParams<T>>& a, int nthreads, size_t lds, hipStream_t s);

template <typename T>
void launch_xfwd(const XFwdParams<T>& p, hipStream_t s);
template <typename T>
void launch_ypass(const YPassParams<T>& p, int inverse, hipStream_t s);
template <typename T>
void launch_zpush(const ZPushParams<T>& p, int nthreads, hipStream_t s);
// The two-stage z kernel for p.ra, p.rb (one of kZTwoStage).
template <typename T>
void launch_zpush_two_stage(const ZPushParams<T>& p, hipStream_t s);
template <typename T>
void launch_xinv(const XInvParams<T>& p, hipStream_t s);

// Tables (FP64 math, stored at working precision).
// Stage-major twiddle table of `sch` (see fft_lds.hpp), n entries allocated.
void launch_twiddles(void* dst, const LineSchedule& sch, int fp64, hipStream_t s);
void launch_bluestein(void* chirp, void* filt, int n, int m, int fp64, hipStream_t s);
void launch_modk(double* dst, int n, int count, double d, int order, int staggered, hipStream_t s);
// kappa = k_s exp(i k d / 2) of each DFT index at working precision (staggered grids).
void launch_shifted(const double* ks, void* dst, int n, int count, int fp64, hipStream_t s);
void launch_coef(void* coef, void* kxw, void* kyw, void* kzw, const double* kx, const double* ky,
                 const double* kz, int NXH, int NY, int NZ, double dt, double c, double norm, int fp64,
                 hipStream_t s);

// Standalone guard fill / merge (element-wise gathers).
void launch_guard_fill(const void* const* g1, void* const* box, int nfields, int esize, const int box_dims[3],
                       const int start[3], const int gdims[3], hipStream_t s);
void launch_guard_merge(const void* const* box, void* const* g1, int nfields, int esize, const int box_dims[3],
                        const int guard[3], const int interior[3], const int origin[3], const int gdims[3],
                        int mode, hipStream_t s);

// Two-step PML element-wise kernels (split parts: set A = parts[0..5], set B = parts[6..11]).
void launch_pml_sum(const void* const* parts, void* const* full, long long ncell, int fp64, hipStream_t s);
void launch_pml_update(void* const* parts, const void* const* inc, const void* const damp[3], int set, int NX,
                       int NY, int NZ, int fp64, hipStream_t s);

// Records a message for psatd_last_error() and returns `code`.
int report_error(int code, const char* fmt, ...);

}  // namespace psatd
