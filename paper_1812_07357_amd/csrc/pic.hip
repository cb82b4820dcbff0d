// Particle side of the PIC cycle around the PSATD step (gfx950): field gather +
// relativistic Boris push, and current / charge deposition through D1 tiles.
//
// arXiv:1812.07357, Sec. 2.5.1 (Fig. 4): particles are pushed with the fields at
// their positions, their current and charge are deposited with linear
// interpolation, Maxwell's equations are solved, and the fields are gathered
// back.  Sec. 2.5.2: particle-mesh work runs on the grid G1 split into
// sub-domains D1 whose guard cells are as wide as the interpolation stencil,
// while the FFTs run on the boxes of G2 (decomposition D2, psatd_step_g1 /
// psatd_batch_*), coupled by guard fill and interior copy.
//
// Here a D1 sub-domain is a tile of T^3 cells of G1 worked on by one workgroup:
// the particles are counted per tile (by their start position), the tile
// offsets scanned, the particles listed per tile, and each workgroup deposits its
// tile's particles into LDS over the tile plus its guard cells (Reach<K>::lo below,
// Reach<K>::hi above, per axis), then adds that LDS block into G1 (the guard cells land
// on the neighbouring tiles' cells: the additive guard merge of the D1
// decomposition).  The guards hold the stencil of a particle that started in
// the tile and moved less than one cell during the step, which the host ensures
// (c dt below the smallest cell size, with a margin for rounding).  The LDS block sums in
// 64-bit fixed point with a power-of-two scale per tile, so a tile's sums are exact and do
// not depend on the order of the atomics.
//
// Weights: a quantity of a component with half-cell offset o sits at grid point
// (i + o/2) d; a particle at x spreads over the (K+1)^3 points around it with the
// product of the 1D centred B-spline weights of degree K (Sec. 2.5.1 allows linear or
// higher-order interpolation: K = 1 cloud in cell, 2 triangular-shaped cloud, 3 cubic),
// and the gather uses the same weights.  rho = q S / (dx dy dz)
// at the start and end positions, J = q v S / (dx dy dz) at the mid-point with
// the half-step velocity.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "../../include/psatd.h"
#include "internal.hpp"

namespace psatd {
namespace {

constexpr int kPicThreads = 256;
// Stencil reach of a particle that starts in cell c and moves less than one cell, for
// weights of degree K: the points of rho_new and of J (mid-point, half a cell away) span
// [c - 1, c + 2] (K = 1) or [c - 2, c + 3] (K = 2, 3).
template <int K>
struct Reach {
  static constexpr int lo = K == 1 ? 1 : 2, hi = K == 1 ? 2 : 3;
};
constexpr int kMaxShape = 3;
// c dt may reach this fraction of the smallest cell (the rest absorbs rounding).
constexpr double kMaxCourant = 0.999;
constexpr int kTileMax = 12;

// half-cell offsets of Ex Ey Ez Bx By Bz Jx Jy Jz rho_old rho_new on the staggered grid
__constant__ int kOffStag[11][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {0, 1, 1}, {1, 0, 1}, {1, 1, 0},
                                    {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {0, 0, 0}, {0, 0, 0}};

template <typename T>
struct PicArgs {
  int gx, gy, gz;
  T dx, dy, dz;   // cell sizes
  T idx, idy, idz;  // 1 / cell sizes
  T lx, ly, lz;   // periodic lengths
  T dt, c, q, qm;
  T inv_vol;
  int stag;
  int tile, tx, ty, tz, ntiles;  // D1 tiles: edge, tiles per axis, total
  int n;
};

// Centred B-spline weights of degree K of coordinate s (in cells): the K + 1 points
// first, ..., first + K and their weights.
template <int K, typename T>
__device__ __forceinline__ void shape1d(T s, int& first, T* w) {
  if constexpr (K == 1) {
    const T f = floor(s), t = s - f;
    first = (int)f;
    w[0] = T(1) - t;
    w[1] = t;
  } else if constexpr (K == 2) {
    const T r = floor(s + T(0.5)), t = s - r;
    first = (int)r - 1;
    w[0] = T(0.5) * (T(0.5) - t) * (T(0.5) - t);
    w[1] = T(0.75) - t * t;
    w[2] = T(0.5) * (T(0.5) + t) * (T(0.5) + t);
  } else {
    const T f = floor(s), t = s - f, t2 = t * t, t3 = t2 * t, u = T(1) - t;
    first = (int)f - 1;
    w[0] = u * u * u / T(6);
    w[1] = (T(4) - T(6) * t2 + T(3) * t3) / T(6);
    w[2] = (T(1) + T(3) * t + T(3) * t2 - T(3) * t3) / T(6);
    w[3] = t3 / T(6);
  }
}


// Index i of an axis of n cells folded into [0, n): positions in [0, L) need at most one
// add or subtract; the clamp keeps out-of-contract positions inside the array.
__device__ __forceinline__ int fold(int i, int n) {
  if (i < 0) i += n;
  if (i >= n) i -= n;
  return min(max(i, 0), n - 1);
}

// The (K+1)^3 G1 points around (x, y, z) (lengths) of a quantity with half-cell offsets
// (ox, oy, oz), periodic G1, as per-axis folded indices and weights.
template <int K, typename T>
struct Points {
  int xs[K + 1], ys[K + 1], zs[K + 1];
  T wx[K + 1], wy[K + 1], wz[K + 1];
};

template <int K, typename T>
__device__ __forceinline__ void grid_points(Points<K, T>& g, const PicArgs<T>& a, T x, T y, T z, int ox, int oy,
                                            int oz) {
  int fx, fy, fz;
  shape1d<K>(x * a.idx - T(0.5) * ox, fx, g.wx);
  shape1d<K>(y * a.idy - T(0.5) * oy, fy, g.wy);
  shape1d<K>(z * a.idz - T(0.5) * oz, fz, g.wz);
#pragma unroll
  for (int c = 0; c <= K; ++c) {
    g.xs[c] = fold(fx + c, a.gx);
    g.ys[c] = fold(fy + c, a.gy) * a.gx;
    g.zs[c] = fold(fz + c, a.gz) * a.gy * a.gx;
  }
}

// K + 1 consecutive values of a row, read with one multi-word load (4-byte aligned vectors)
template <int K, typename T>
struct RowRun {
  T v[K + 1];
};
template <int K, typename T>
__device__ __forceinline__ RowRun<K, T> load_run(const T* p) {
  typedef T vec_t __attribute__((ext_vector_type(K + 1), aligned(alignof(T))));
  const vec_t x = *reinterpret_cast<const vec_t*>(p);
  RowRun<K, T> r;
#pragma unroll
  for (int c = 0; c <= K; ++c) r.v[c] = x[c];
  return r;
}

template <int K, typename T>
__device__ __forceinline__ T gather_at(const T* __restrict__ f, const Points<K, T>& g) {
  T acc = 0;
  // the x points are consecutive unless the stencil wraps around the periodic edge
  const bool run = g.xs[K] == g.xs[0] + K;
#pragma unroll
  for (int cz = 0; cz <= K; ++cz)
#pragma unroll
    for (int cy = 0; cy <= K; ++cy) {
      const T wyz = g.wy[cy] * g.wz[cz];
      const T* row = f + g.zs[cz] + g.ys[cy];
      RowRun<K, T> r;
      if (run) {
        r = load_run<K>(row + g.xs[0]);
      } else {
#pragma unroll
        for (int cx = 0; cx <= K; ++cx) r.v[cx] = row[g.xs[cx]];
      }
#pragma unroll
      for (int cx = 0; cx <= K; ++cx) acc += r.v[cx] * (g.wx[cx] * wyz);
    }
  return acc;
}

template <typename T>
struct PushPtrs {
  const T* f[6];  // Ex Ey Ez Bx By Bz on G1
  T* x[3];
  T* u[3];
  T* x_old[3];
};

// Gather E, B at x, relativistic Boris push of u = gamma v, x moved by dt u / gamma (wrapped).
// STAG: staggered grid (each component at its own half-cell offsets); otherwise the six
// components share one set of points and weights.
template <typename T, bool STAG, int K>
__global__ void __launch_bounds__(kPicThreads) k_pic_push(PicArgs<T> a, PushPtrs<T> p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  // the particle arrays stream through once (non-temporal), which leaves the caches to the
  // field rows that neighbouring particles gather again
  const T x = __builtin_nontemporal_load(&p.x[0][i]), y = __builtin_nontemporal_load(&p.x[1][i]),
          z = __builtin_nontemporal_load(&p.x[2][i]);
  T E[3], B[3];
  Points<K, T> g;
  if constexpr (K > 1) {
    // one field at a time (a loop that is not unrolled), so that the (K+1)^3 loads of one
    // field are in flight together without the registers of all six
    T eb[6];
    if constexpr (!STAG) grid_points<K>(g, a, x, y, z, 0, 0, 0);
#pragma unroll 1
    for (int k = 0; k < 6; ++k) {
      if constexpr (STAG) {
        // E_a half a cell up along a; B_a along the two other axes
        const int c = k < 3 ? k : k - 3;
        const bool e = k < 3;
        grid_points<K>(g, a, x, y, z, (c == 0) == e, (c == 1) == e, (c == 2) == e);
      }
      const T v = gather_at<K>(p.f[k], g);
#pragma unroll
      for (int j = 0; j < 6; ++j)
        if (j == k) eb[j] = v;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      E[c] = eb[c];
      B[c] = eb[3 + c];
    }
  } else if constexpr (STAG) {
    // E_a half a cell up along a; B_a along the two other axes
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      grid_points<K>(g, a, x, y, z, k == 0, k == 1, k == 2);
      E[k] = gather_at<K>(p.f[k], g);
      grid_points<K>(g, a, x, y, z, k != 0, k != 1, k != 2);
      B[k] = gather_at<K>(p.f[3 + k], g);
    }
  } else {
    grid_points<K>(g, a, x, y, z, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      E[k] = gather_at<K>(p.f[k], g);
      B[k] = gather_at<K>(p.f[3 + k], g);
    }
  }
  const T h = T(0.5) * a.qm * a.dt;
  const T ic2 = T(1) / (a.c * a.c);
  T um[3] = {__builtin_nontemporal_load(&p.u[0][i]) + h * E[0], __builtin_nontemporal_load(&p.u[1][i]) + h * E[1],
             __builtin_nontemporal_load(&p.u[2][i]) + h * E[2]};
  const T gm = sqrt(T(1) + (um[0] * um[0] + um[1] * um[1] + um[2] * um[2]) * ic2);
  const T t[3] = {h * B[0] / gm, h * B[1] / gm, h * B[2] / gm};
  const T t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  const T s[3] = {T(2) * t[0] / (T(1) + t2), T(2) * t[1] / (T(1) + t2), T(2) * t[2] / (T(1) + t2)};
  const T up[3] = {um[0] + um[1] * t[2] - um[2] * t[1], um[1] + um[2] * t[0] - um[0] * t[2],
                   um[2] + um[0] * t[1] - um[1] * t[0]};
  const T un[3] = {um[0] + up[1] * s[2] - up[2] * s[1] + h * E[0], um[1] + up[2] * s[0] - up[0] * s[2] + h * E[1],
                   um[2] + up[0] * s[1] - up[1] * s[0] + h * E[2]};
  const T gn = sqrt(T(1) + (un[0] * un[0] + un[1] * un[1] + un[2] * un[2]) * ic2);
  const T L[3] = {a.lx, a.ly, a.lz};
  const T xs[3] = {x, y, z};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T xn = xs[k] + a.dt * un[k] / gn;
    xn -= L[k] * floor(xn / L[k]);
    if (xn >= L[k]) xn -= L[k];  // rounding at the upper edge
    __builtin_nontemporal_store(xs[k], &p.x_old[k][i]);
    __builtin_nontemporal_store(xn, &p.x[k][i]);
    __builtin_nontemporal_store(un[k], &p.u[k][i]);
  }
}

// D1 tile of a start position.
template <typename T>
__device__ __forceinline__ int tile_of(const PicArgs<T>& a, T x, T y, T z) {
  // clamped, so that a position outside [0, L) cannot index past the tile arrays
  const int cx = min(max((int)(x * a.idx), 0), a.gx - 1), cy = min(max((int)(y * a.idy), 0), a.gy - 1),
            cz = min(max((int)(z * a.idz), 0), a.gz - 1);
  return ((cz / a.tile) * a.ty + cy / a.tile) * a.tx + cx / a.tile;
}

template <typename T>
struct DepPtrs {
  const T* xo[3];
  const T* xn[3];
  const T* u[3];
  T* g[5];  // Jx Jy Jz rho_old rho_new on G1
  int* count;   // ntiles
  int* offset;  // ntiles + 1
  int* cursor;  // ntiles
  int* list;    // n particle indices, tile by tile
};

__global__ void k_zero_int(int* a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

template <typename T>
__global__ void k_zero_fields(DepPtrs<T> p, long long ncell) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ncell)
#pragma unroll
    for (int f = 0; f < 5; ++f) p.g[f][i] = T(0);
}

// Runs of equal keys in consecutive lanes of a wave: whether this lane leads its run,
// the run's leading lane and (at the leader) its length.  Inactive lanes carry
// distinct keys, so they never join a run.  Every lane of the wave must call it.
struct WaveRun {
  bool head;
  int leader, len;
};
__device__ __forceinline__ WaveRun wave_run(int key, bool active) {
  const int lane = __lane_id();
  const int k = active ? key : -1 - lane;
  const int prev = __shfl_up(k, 1);
  const bool head = lane == 0 || prev != k;
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = (2ull << lane) - 1ull;  // lanes 0..lane (all for lane 63)
  const unsigned long long after = heads & ~upto;
  WaveRun r;
  r.head = head;
  r.leader = 63 - __clzll(heads & upto);
  r.len = (after ? __ffsll((long long)after) - 1 : 64) - lane;
  return r;
}

// Particles per D1 tile; particles of one tile in consecutive lanes (cell-ordered
// input) add their count with one atomic per run.
template <typename T>
__global__ void __launch_bounds__(kPicThreads) k_tile_count(PicArgs<T> a, DepPtrs<T> p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = i < a.n;
  const int t = active ? tile_of(a, p.xo[0][i], p.xo[1][i], p.xo[2][i]) : 0;
  const WaveRun r = wave_run(t, active);
  if (active && r.head) atomicAdd(&p.count[t], r.len);
}

// Exclusive scan of the tile counts by one workgroup (offset[ntiles] = n); cursors start
// at the offsets.
__global__ void __launch_bounds__(1024) k_tile_scan(const int* count, int* offset, int* cursor, int ntiles) {
  __shared__ int part[1024];
  const int tid = threadIdx.x, nth = blockDim.x;
  const int per = (ntiles + nth - 1) / nth;
  const int lo = min(ntiles, tid * per), hi = min(ntiles, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += count[i];
  part[tid] = s;
  __syncthreads();
  for (int d = 1; d < nth; d <<= 1) {  // inclusive scan of the per-thread sums
    const int v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = part[tid] - s;
  for (int i = lo; i < hi; ++i) {
    offset[i] = run;
    cursor[i] = run;
    run += count[i];
  }
  if (tid == nth - 1) offset[ntiles] = part[nth - 1];
}

// Particle indices listed tile by tile: a run of one tile's particles in consecutive
// lanes takes its slots with one atomic and fills them in lane order.
template <typename T>
__global__ void __launch_bounds__(kPicThreads) k_tile_list(PicArgs<T> a, DepPtrs<T> p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = i < a.n;
  const int t = active ? tile_of(a, p.xo[0][i], p.xo[1][i], p.xo[2][i]) : 0;
  const WaveRun r = wave_run(t, active);
  int base = 0;
  if (active && r.head) base = atomicAdd(&p.cursor[t], r.len);
  base = __shfl(base, r.leader);
  if (active) p.list[base + (int)__lane_id() - r.leader] = i;
}

// The stencil of one quantity of one particle inside the LDS block of a tile, in
// separable form: the block-local index of its first point and the 1D weights per axis
// (the value folded into the x weights).  The block spans E = T + Reach<K>::lo +
// Reach<K>::hi cells per axis from the tile's first cell (bx, by, bz) minus Reach<K>::lo.
template <int K, typename T>
struct Axes {
  int l0;
  T wx[K + 1], wy[K + 1], wz[K + 1];
};

template <int K, typename T>
__device__ __forceinline__ void stencil_axes(Axes<K, T>& s, int E, const PicArgs<T>& a, int slot, T x, T y, T z,
                                             T value, int bx, int by, int bz) {
  const int ox = a.stag ? kOffStag[slot][0] : 0, oy = a.stag ? kOffStag[slot][1] : 0,
            oz = a.stag ? kOffStag[slot][2] : 0;
  int ix, iy, iz;
  shape1d<K>(x * a.idx - T(0.5) * ox, ix, s.wx);
  shape1d<K>(y * a.idy - T(0.5) * oy, iy, s.wy);
  shape1d<K>(z * a.idz - T(0.5) * oz, iz, s.wz);
#pragma unroll
  for (int c = 0; c <= K; ++c) s.wx[c] *= value;
  // local indices relative to the block origin (tile origin - guard); positions near the
  // periodic edge are taken on the tile's side of the edge.  For positions in [0, L) whose
  // particle started in the tile the first point lies in [0, E - 1 - K]; the clamp only
  // keeps positions that break that contract inside the block.
  auto local = [&](int i, int b, int n) {
    int l = i - (b - Reach<K>::lo);
    if (l < 0) l += n;
    if (l >= n) l -= n;
    return min(max(l, 0), E - 1 - K);
  };
  s.l0 = (local(iz, bz, a.gz) * E + local(iy, by, a.gy)) * E + local(ix, bx, a.gx);
}

// The linear stencil as eight weighted values, corners in (z, y, x) order: the form the
// run accumulation below sums in registers.
template <typename T>
struct Stencil {
  int l0;
  T w[8];
};

template <typename T>
__device__ __forceinline__ void stencil(Stencil<T>& s, int E, const PicArgs<T>& a, int slot, T x, T y, T z,
                                        T value, int bx, int by, int bz) {
  Axes<1, T> g;
  stencil_axes<1>(g, E, a, slot, x, y, z, value, bx, by, bz);
  s.l0 = g.l0;
#pragma unroll
  for (int c = 0; c < 8; ++c) s.w[c] = g.wx[c & 1] * (g.wy[(c >> 1) & 1] * g.wz[c >> 2]);
}

// The LDS block accumulates in 64-bit fixed point: each weighted value times a power of two
// `scale`, rounded to an integer, added with an integer LDS atomic (floating-point LDS
// atomics are several times slower).  Integer sums are exact and independent of their order;
// the scale keeps every sum below 2^62 in magnitude (see k_deposit_tiles).
using fixed_t = unsigned long long;

template <typename T>
__device__ __forceinline__ void stencil_add(fixed_t* blk, int E, const Stencil<T>& s, T scale) {
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const long long v = llrint((double)(s.w[c] * scale));
    atomicAdd(&blk[s.l0 + ((c >> 2) * E + ((c >> 1) & 1)) * E + (c & 1)], (fixed_t)v);
  }
}

// A stencil of degree K > 1 straight into the block, (K + 1)^3 atomics (its weights do not
// fit a register run).
template <int K, typename T>
__device__ __forceinline__ void stencil_add_axes(fixed_t* blk, int E, const Axes<K, T>& s, T scale) {
#pragma unroll
  for (int cz = 0; cz <= K; ++cz)
#pragma unroll
    for (int cy = 0; cy <= K; ++cy) {
      const T wyz = s.wy[cy] * s.wz[cz] * scale;
      fixed_t* row = blk + s.l0 + (cz * E + cy) * E;
#pragma unroll
      for (int cx = 0; cx <= K; ++cx) atomicAdd(&row[cx], (fixed_t)llrint((double)(s.wx[cx] * wyz)));
    }
}

// Running sum of the stencils of consecutive particles of one thread: particles whose
// stencil has the same lower corner are summed in registers, and the LDS block receives one
// set of atomics per run (particles of one cell come in runs when the input is cell-ordered).
template <typename T>
__device__ __forceinline__ void stencil_run(fixed_t* blk, int E, Stencil<T>& acc, const Stencil<T>& cur, T scale) {
  if (cur.l0 == acc.l0) {
#pragma unroll
    for (int c = 0; c < 8; ++c) acc.w[c] += cur.w[c];
  } else {
    if (acc.l0 >= 0) stencil_add(blk, E, acc, scale);
    acc = cur;
  }
}

// One workgroup per D1 tile: its particles' J (mid-point), rho_old (start) and rho_new
// (end) into LDS over the tile and its guard cells, then the block either added into G1
// with global atomics (blocks == nullptr) or stored whole, tile by tile, into `blocks`
// ([tile][quantity][z][y][x], E^3 values per quantity) for k_gather_blocks.
template <typename T, int K>
__global__ void __launch_bounds__(kPicThreads) k_deposit_tiles(PicArgs<T> a, DepPtrs<T> p, T* __restrict__ blocks) {
  extern __shared__ double2 pic_smem[];
  fixed_t* lds = reinterpret_cast<fixed_t*>(pic_smem);
  constexpr int GL = Reach<K>::lo;
  const int E = a.tile + GL + Reach<K>::hi;
  const int ncl = E * E * E;
  const int tid = threadIdx.x;
  // merge walk: thread (row r0, column lx) of R = blockDim / E rows per round
  const int R = blockDim.x / E, r0 = tid / E, lx = tid - r0 * E;
  const int dy = R % E, dz = (R / E) % E, df = R / (E * E);
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const int tz = t / (a.tx * a.ty), rem = t - tz * a.tx * a.ty, ty = rem / a.tx, tx = rem - ty * a.tx;
    const int bx = tx * a.tile, by = ty * a.tile, bz = tz * a.tile;
    for (int i = tid; i < 5 * ncl; i += blockDim.x) lds[i] = 0;
    __syncthreads();
    const T ic2 = T(1) / (a.c * a.c);
    const T qv = a.q * a.inv_vol;
    // each thread takes a contiguous run of the tile's list, so the lanes of a wave work in
    // different cells (no two lanes add to one LDS word in the same instruction) and one
    // thread's consecutive particles share stencils
    const int first = p.offset[t], count = p.offset[t + 1] - first;
    // fixed-point scales of J and rho: a particle adds at most |q| c / V (|v| < c) to a J
    // point and |q| / V to a rho point, so with count particles every sum stays below
    // count * bound * scale < 2^62.  Powers of two: scaling and unscaling are exact.
    const double bq = fabs((double)a.q) * (double)a.inv_vol * (double)max(count, 1);
    const int ej = 61 - ilogb(fmax(bq * (double)a.c * 1.0000001, 1e-300));
    const int er = 61 - ilogb(fmax(bq * 1.0000001, 1e-300));
    // (capped where the bound is tiny: then bound * 2^120 is below 2^62 anyway)
    const int ejc = min(ej, 120), erc = min(er, 120);
    const T sj = (T)ldexp(1.0, ejc), sr = (T)ldexp(1.0, erc);
    const int per = (count + (int)blockDim.x - 1) / (int)blockDim.x;
    const int e0 = first + min(count, tid * per), e1 = first + min(count, (tid + 1) * per);
    Stencil<T> acc[K == 1 ? 5 : 1], cur;
#pragma unroll
    for (int q = 0; q < (K == 1 ? 5 : 1); ++q) acc[q].l0 = -1;
    for (int e = e0; e < e1; ++e) {
      const int i = p.list[e];
      const T u0 = p.u[0][i], u1 = p.u[1][i], u2 = p.u[2][i];
      const T ig = T(1) / sqrt(T(1) + (u0 * u0 + u1 * u1 + u2 * u2) * ic2);
      const T v[3] = {u0 * ig, u1 * ig, u2 * ig};
      const T x0 = p.xo[0][i], y0 = p.xo[1][i], z0 = p.xo[2][i];
      // mid-point (unwrapped from the start position; stencil() folds the periodic edge)
      T xm = x0 + T(0.5) * a.dt * v[0], ym = y0 + T(0.5) * a.dt * v[1], zm = z0 + T(0.5) * a.dt * v[2];
      xm -= a.lx * floor(xm / a.lx);
      ym -= a.ly * floor(ym / a.ly);
      zm -= a.lz * floor(zm / a.lz);
      if constexpr (K == 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          stencil(cur, E, a, 6 + k, xm, ym, zm, qv * v[k], bx, by, bz);
          stencil_run(lds + k * ncl, E, acc[k], cur, sj);
        }
        stencil(cur, E, a, 9, x0, y0, z0, qv, bx, by, bz);
        stencil_run(lds + 3 * ncl, E, acc[3], cur, sr);
        stencil(cur, E, a, 10, p.xn[0][i], p.xn[1][i], p.xn[2][i], qv, bx, by, bz);
        stencil_run(lds + 4 * ncl, E, acc[4], cur, sr);
      } else {
        Axes<K, T> g;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          stencil_axes<K>(g, E, a, 6 + k, xm, ym, zm, qv * v[k], bx, by, bz);
          stencil_add_axes<K>(lds + k * ncl, E, g, sj);
        }
        stencil_axes<K>(g, E, a, 9, x0, y0, z0, qv, bx, by, bz);
        stencil_add_axes<K>(lds + 3 * ncl, E, g, sr);
        stencil_axes<K>(g, E, a, 10, p.xn[0][i], p.xn[1][i], p.xn[2][i], qv, bx, by, bz);
        stencil_add_axes<K>(lds + 4 * ncl, E, g, sr);
      }
    }
    if constexpr (K == 1) {
#pragma unroll
      for (int q = 0; q < 5; ++q)
        if (acc[q].l0 >= 0) stencil_add(lds + q * ncl, E, acc[q], q < 3 ? sj : sr);
    }
    __syncthreads();
    if (blocks) {
      // the whole block, unscaled, in the tile's slot (consecutive threads, consecutive words)
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        const double sc = ldexp(1.0, -(f < 3 ? ejc : erc));
        T* dst = blocks + ((long long)t * 5 + f) * ncl;
        for (int i = tid; i < ncl; i += blockDim.x) dst[i] = (T)((double)(long long)lds[f * ncl + i] * sc);
      }
    } else if (r0 < R) {
      // the block (tile and guards) added into G1: guard cells are the neighbours' cells.
      // Rows (f, z, y) are walked with carries, so no element needs a division.
      auto wrap_near = [](int v, int n) {  // v in [-n, ...): one add or subtract except on tiny grids
        if (v < 0) v += n;
        if (v >= n) {
          v -= n;
          if (v >= n) v %= n;
        }
        return v;
      };
      const int gxi = wrap_near(bx - GL + lx, a.gx);
      int y = r0 % E, z = (r0 / E) % E, f = r0 / (E * E);
      while (f < 5) {
        const long long iv = (long long)lds[((f * E + z) * E + y) * E + lx];
        if (iv != 0) {
          const T v = (T)((double)iv * ldexp(1.0, -(f < 3 ? ejc : erc)));
          const int gyi = wrap_near(by - GL + y, a.gy), gzi = wrap_near(bz - GL + z, a.gz);
          unsafeAtomicAdd(&p.g[f][((long long)gzi * a.gy + gyi) * a.gx + gxi], v);
        }
        y += dy;
        if (y >= E) {
          y -= E;
          ++z;
        }
        z += dz;
        if (z >= E) {
          z -= E;
          ++f;
        }
        f += df;
      }
    }
    __syncthreads();
  }
}

// The blocks stored by k_deposit_tiles summed into G1: one workgroup per tile, one thread
// per cell of the tile (x fastest), so that a wave reads rows of several block rows at once.
// A cell lies in the block of its own tile and, within Reach<K>::hi cells of the tile's
// lower face or Reach<K>::lo cells of its upper face, in the block of the neighbour across
// it.  Requires tiles that divide the grid, at least two tiles per axis and guards no wider
// than a tile, so that along each axis a cell is reached by its own tile and at most one
// neighbour (with two tiles per axis both neighbours are the same tile, reached through one
// face or the other).  Every cell is written (no zeroing first), with a fixed order of the
// sums.
template <typename T, int K>
__global__ void __launch_bounds__(256) k_gather_blocks(PicArgs<T> a, DepPtrs<T> p, const T* __restrict__ blocks) {
  constexpr int GL = Reach<K>::lo, GH = Reach<K>::hi;
  const int T_ = a.tile, E = T_ + GL + GH, T2 = T_ * T_;
  const long long ncl = (long long)E * E * E;
  const int tile = blockIdx.x;
  const int tz = tile / (a.tx * a.ty), ty = (tile - tz * a.tx * a.ty) / a.tx, tx = tile - (tz * a.ty + ty) * a.tx;
  // per axis: the tiles whose block covers local cell c, and the cell's index in each
  auto reach = [&](int c, int t, int nt, int* ts, int* ls) {
    ts[0] = t;
    ls[0] = c + GL;
    int m = 1;
    if (c < GH) {  // in the upper guard of the tile below
      ts[m] = t == 0 ? nt - 1 : t - 1;
      ls[m] = c + T_ + GL;
      ++m;
    } else if (c >= T_ - GL) {  // in the lower guard of the tile above
      ts[m] = t == nt - 1 ? 0 : t + 1;
      ls[m] = c - T_ + GL;
      ++m;
    }
    return m;
  };
  for (int q = threadIdx.x; q < T2 * T_; q += blockDim.x) {
    const int lz = q / T2, ly = (q - lz * T2) / T_, lx = q - lz * T2 - ly * T_;
    int tsx[2], lsx[2], tsy[2], lsy[2], tsz[2], lsz[2];
    const int mx = reach(lx, tx, a.tx, tsx, lsx), my = reach(ly, ty, a.ty, tsy, lsy),
              mz = reach(lz, tz, a.tz, tsz, lsz);
    T acc[5] = {0, 0, 0, 0, 0};
    for (int iz = 0; iz < mz; ++iz)
      for (int iy = 0; iy < my; ++iy)
        for (int ix = 0; ix < mx; ++ix) {
          const long long t = ((long long)tsz[iz] * a.ty + tsy[iy]) * a.tx + tsx[ix];
          const T* b = blocks + t * 5 * ncl + ((long long)lsz[iz] * E + lsy[iy]) * E + lsx[ix];
#pragma unroll
          for (int f = 0; f < 5; ++f) acc[f] += b[f * ncl];
        }
    const long long cell = ((long long)(tz * T_ + lz) * a.gy + (ty * T_ + ly)) * a.gx + (tx * T_ + lx);
#pragma unroll
    for (int f = 0; f < 5; ++f) p.g[f][cell] = acc[f];
  }
}

}  // namespace
}  // namespace psatd

using namespace psatd;

struct psatd_pic {
  psatd_pic_desc d{};
  int fp64 = 0;
  int tx = 0, ty = 0, tz = 0, ntiles = 0;
  int* count = nullptr;
  int* offset = nullptr;
  int* cursor = nullptr;
  int* list = nullptr;
  void* blocks = nullptr;  // per-tile deposit blocks (NULL: blocks merged with atomics)
};

namespace {

template <typename T>
PicArgs<T> pic_args(const psatd_pic* o, int n) {
  PicArgs<T> a{};
  const psatd_pic_desc& d = o->d;
  a.gx = d.gx;
  a.gy = d.gy;
  a.gz = d.gz;
  a.dx = T(d.dx);
  a.dy = T(d.dy);
  a.dz = T(d.dz);
  a.idx = T(1.0 / d.dx);
  a.idy = T(1.0 / d.dy);
  a.idz = T(1.0 / d.dz);
  a.lx = T(d.gx * d.dx);
  a.ly = T(d.gy * d.dy);
  a.lz = T(d.gz * d.dz);
  a.dt = T(d.dt);
  a.c = T(d.c);
  a.q = T(d.q);
  a.qm = T(d.q_over_m);
  a.inv_vol = T(1.0 / (d.dx * d.dy * d.dz));
  a.stag = (d.flags & PSATD_FLAG_STAGGERED) ? 1 : 0;
  a.tile = d.tile;
  a.tx = o->tx;
  a.ty = o->ty;
  a.tz = o->tz;
  a.ntiles = o->ntiles;
  a.n = n;
  return a;
}

// LDS of one deposit workgroup: five fixed-point quantities over the tile and its guard
// cells, for particle shapes of degree `shape`.
size_t pic_lds_bytes(int tile, int shape) {
  const size_t e = (size_t)tile + (shape == 1 ? Reach<1>::lo + Reach<1>::hi : Reach<2>::lo + Reach<2>::hi);
  return 5 * e * e * e * sizeof(fixed_t);
}

// degree of the particle shape of a descriptor (0 means linear)
int shape_of(const psatd_pic_desc& d) { return d.shape == 0 ? 1 : d.shape; }

unsigned blocks_for(long long n, int th) { return (unsigned)((n + th - 1) / th); }

template <typename T>
int pic_push(psatd_pic* o, void* const* g1, void* const* x, void* const* u, void* const* x_old, int n,
             hipStream_t s) {
  if (n == 0) return PSATD_OK;
  PushPtrs<T> p{};
  for (int k = 0; k < 6; ++k) p.f[k] = (const T*)g1[k];
  for (int k = 0; k < 3; ++k) {
    p.x[k] = (T*)x[k];
    p.u[k] = (T*)u[k];
    p.x_old[k] = (T*)x_old[k];
  }
  const PicArgs<T> a = pic_args<T>(o, n);
  const dim3 grid(blocks_for(n, kPicThreads)), block(kPicThreads);
  switch (shape_of(o->d) * 2 + a.stag) {
    case 2: hipLaunchKernelGGL((k_pic_push<T, false, 1>), grid, block, 0, s, a, p); break;
    case 3: hipLaunchKernelGGL((k_pic_push<T, true, 1>), grid, block, 0, s, a, p); break;
    case 4: hipLaunchKernelGGL((k_pic_push<T, false, 2>), grid, block, 0, s, a, p); break;
    case 5: hipLaunchKernelGGL((k_pic_push<T, true, 2>), grid, block, 0, s, a, p); break;
    case 6: hipLaunchKernelGGL((k_pic_push<T, false, 3>), grid, block, 0, s, a, p); break;
    default: hipLaunchKernelGGL((k_pic_push<T, true, 3>), grid, block, 0, s, a, p); break;
  }
  return PSATD_OK;
}

template <typename T, int K>
void launch_deposit(const PicArgs<T>& a, const DepPtrs<T>& p, T* blocks, size_t lds, hipStream_t s) {
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)k_deposit_tiles<T, K>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  // one tile per workgroup (the loop inside covers grids beyond the cap)
  const unsigned grid = (unsigned)std::min(a.ntiles, 1 << 20);
  hipLaunchKernelGGL((k_deposit_tiles<T, K>), dim3(grid), dim3(kPicThreads), lds, s, a, p, blocks);
  if (blocks) hipLaunchKernelGGL((k_gather_blocks<T, K>), dim3(a.ntiles), dim3(256), 0, s, a, p, (const T*)blocks);
}

template <typename T>
int pic_deposit(psatd_pic* o, void* const* g1, const void* const* x_old, const void* const* x, const void* const* u,
                int n, hipStream_t s) {
  DepPtrs<T> p{};
  for (int k = 0; k < 3; ++k) {
    p.xo[k] = (const T*)x_old[k];
    p.xn[k] = (const T*)x[k];
    p.u[k] = (const T*)u[k];
  }
  for (int f = 0; f < 5; ++f) p.g[f] = (T*)g1[6 + f];
  p.count = o->count;
  p.offset = o->offset;
  p.cursor = o->cursor;
  p.list = o->list;
  const PicArgs<T> a = pic_args<T>(o, n);
  const long long ncell = (long long)o->d.gx * o->d.gy * o->d.gz;
  T* blocks = (T*)o->blocks;
  // with per-tile blocks every cell is written by the gather; otherwise the atomics add
  // into zeroed arrays
  if (!blocks || n == 0) hipLaunchKernelGGL(k_zero_fields<T>, dim3(blocks_for(ncell, 256)), dim3(256), 0, s, p, ncell);
  if (n == 0) return PSATD_OK;
  hipLaunchKernelGGL(k_zero_int, dim3(blocks_for(o->ntiles, 256)), dim3(256), 0, s, o->count, o->ntiles);
  hipLaunchKernelGGL(k_tile_count<T>, dim3(blocks_for(n, kPicThreads)), dim3(kPicThreads), 0, s, a, p);
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, s, o->count, o->offset, o->cursor, o->ntiles);
  hipLaunchKernelGGL(k_tile_list<T>, dim3(blocks_for(n, kPicThreads)), dim3(kPicThreads), 0, s, a, p);
  const int shape = shape_of(o->d);
  const size_t lds = pic_lds_bytes(o->d.tile, shape);
  if (shape == 1)
    launch_deposit<T, 1>(a, p, blocks, lds, s);
  else if (shape == 2)
    launch_deposit<T, 2>(a, p, blocks, lds, s);
  else
    launch_deposit<T, 3>(a, p, blocks, lds, s);
  return PSATD_OK;
}

}  // namespace

extern "C" {

int psatd_pic_create(const psatd_pic_desc* d, psatd_pic** out) {
  if (!out) return report_error(PSATD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d) return report_error(PSATD_EINVAL, "descriptor is NULL");
  if (d->gx <= 0 || d->gy <= 0 || d->gz <= 0) return report_error(PSATD_EINVAL, "grid sizes must be positive");
  if (!(d->dx > 0) || !(d->dy > 0) || !(d->dz > 0) || !(d->dt > 0) || !(d->c > 0))
    return report_error(PSATD_EINVAL, "cell sizes, dt and c must be > 0");
  if (d->precision != PSATD_FP32 && d->precision != PSATD_FP64) return report_error(PSATD_EINVAL, "unknown precision");
  if (d->flags & ~PSATD_FLAG_STAGGERED) return report_error(PSATD_EINVAL, "unknown flags 0x%x", d->flags);
  if (d->tile < 1 || d->tile > kTileMax) return report_error(PSATD_EINVAL, "tile must be in [1, %d]", kTileMax);
  if (d->max_particles < 0) return report_error(PSATD_EINVAL, "max_particles must be >= 0");
  if (d->shape < 0 || d->shape > kMaxShape)
    return report_error(PSATD_EINVAL, "shape must be 0 (linear), 1, 2 or %d", kMaxShape);
  // a particle moves less than c dt per step; the margin covers the rounding of positions
  if (d->c * d->dt > kMaxCourant * std::min(d->dx, std::min(d->dy, d->dz)))
    return report_error(PSATD_EUNSUPPORTED,
                        "c dt = %g exceeds %g of the smallest cell size: a particle could leave its tile's guard "
                        "cells", d->c * d->dt, kMaxCourant);
  if ((double)d->gx * d->gy * d->gz >= 2147483647.0) return report_error(PSATD_EUNSUPPORTED, "grid too large");
  {
    int dev = 0, lim = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lim <= 0) {
      (void)hipGetLastError();
      lim = 64 * 1024;
    }
    const size_t need = pic_lds_bytes(d->tile, shape_of(*d));
    if (need > (size_t)lim)
      return report_error(PSATD_EUNSUPPORTED, "tile %d with shape degree %d needs %zu bytes of LDS per workgroup "
                          "(limit %d)", d->tile, shape_of(*d), need, lim);
  }
  psatd_pic* o = new psatd_pic;
  o->d = *d;
  o->fp64 = d->precision == PSATD_FP64;
  o->tx = (d->gx + d->tile - 1) / d->tile;
  o->ty = (d->gy + d->tile - 1) / d->tile;
  o->tz = (d->gz + d->tile - 1) / d->tile;
  o->ntiles = o->tx * o->ty * o->tz;
  const size_t bytes[4] = {(size_t)o->ntiles * 4, (size_t)(o->ntiles + 1) * 4, (size_t)o->ntiles * 4,
                           (size_t)std::max(1, d->max_particles) * 4};
  int** ptrs[4] = {&o->count, &o->offset, &o->cursor, &o->list};
  for (int k = 0; k < 4; ++k)
    if (hipMalloc((void**)ptrs[k], bytes[k]) != hipSuccess) {
      (void)hipGetLastError();
      for (int j = 0; j < k; ++j) (void)hipFree(*ptrs[j]);
      delete o;
      return report_error(PSATD_ENOMEM, "particle workspace allocation failed");
    }
  // Per-tile blocks for the atomic-free merge (see k_gather_blocks) for shapes of degree 2
  // and 3, where the tiling allows it: their blocks hold 13^3 cells per 8^3 tile, and
  // storing and gathering them beats adding them with global atomics.  For degree 1 (11^3
  // cells per 8^3 tile) the atomics are faster.  Without the memory the blocks are merged
  // with atomics.
  {
    const int shape = shape_of(*d), T = d->tile;
    const int reach = Reach<2>::lo + Reach<2>::hi;
    const bool tiled = shape >= 2 && d->gx % T == 0 && d->gy % T == 0 && d->gz % T == 0 && o->tx >= 2 &&
                       o->ty >= 2 && o->tz >= 2 && reach <= T;
    if (tiled) {
      const size_t e = (size_t)T + reach;
      const size_t b = (size_t)o->ntiles * 5 * e * e * e * (o->fp64 ? sizeof(double) : sizeof(float));
      if (hipMalloc(&o->blocks, b) != hipSuccess) {
        (void)hipGetLastError();
        o->blocks = nullptr;
      }
    }
  }
  *out = o;
  return PSATD_OK;
}

void psatd_pic_destroy(psatd_pic* o) {
  if (!o) return;
  for (int* q : {o->count, o->offset, o->cursor, o->list})
    if (q) (void)hipFree(q);
  if (o->blocks) (void)hipFree(o->blocks);
  delete o;
}

int psatd_pic_push(psatd_pic* o, void* const* g1, void* const* x, void* const* u, void* const* x_old, int n,
                   void* stream) {
  if (!o || !g1 || !x || !u || !x_old) return report_error(PSATD_EINVAL, "NULL argument");
  if (n < 0 || n > o->d.max_particles) return report_error(PSATD_EINVAL, "n = %d outside [0, max_particles]", n);
  if (n == 0) return PSATD_OK;
  for (int k = 0; k < 6; ++k)
    if (!g1[k]) return report_error(PSATD_EINVAL, "field pointer %d is NULL", k);
  for (int k = 0; k < 3; ++k)
    if (!x[k] || !u[k] || !x_old[k]) return report_error(PSATD_EINVAL, "particle array %d is NULL", k);
  const int rc = o->fp64 ? pic_push<double>(o, g1, x, u, x_old, n, (hipStream_t)stream)
                         : pic_push<float>(o, g1, x, u, x_old, n, (hipStream_t)stream);
  if (rc) return rc;
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PSATD_OK : report_error(PSATD_EHIP, "psatd_pic_push: %s", hipGetErrorString(e));
}

int psatd_pic_deposit(psatd_pic* o, void* const* g1, const void* const* x_old, const void* const* x,
                      const void* const* u, int n, void* stream) {
  if (!o || !g1 || !x_old || !x || !u) return report_error(PSATD_EINVAL, "NULL argument");
  if (n < 0 || n > o->d.max_particles) return report_error(PSATD_EINVAL, "n = %d outside [0, max_particles]", n);
  for (int k = 6; k < 11; ++k)
    if (!g1[k]) return report_error(PSATD_EINVAL, "field pointer %d is NULL", k);
  for (int k = 0; n > 0 && k < 3; ++k)
    if (!x[k] || !u[k] || !x_old[k]) return report_error(PSATD_EINVAL, "particle array %d is NULL", k);
  const int rc = o->fp64 ? pic_deposit<double>(o, g1, x_old, x, u, n, (hipStream_t)stream)
                         : pic_deposit<float>(o, g1, x_old, x, u, n, (hipStream_t)stream);
  if (rc) return rc;
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PSATD_OK : report_error(PSATD_EHIP, "psatd_pic_deposit: %s", hipGetErrorString(e));
}

}  // extern "C"
