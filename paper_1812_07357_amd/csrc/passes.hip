// The five passes of one PSATD step on a box (gfx950).
//
//   P1 xfwd   G1 (periodic gather, guard fill fused) or box reals -> x R2C -> layout A
//   P2 ypass  layout A -> y C2C forward -> layout B
//   P3 zpush  layout B -> z C2C forward, analytic push, z C2C inverse -> layout B (E, B)
//   P4 ypass  layout B -> y C2C inverse -> layout A (E, B)
//   P5 xinv   layout A -> x C2R -> box reals or G1 interior (guard merge fused)
//
// Sec. 1.1 of arXiv:1812.07357 (Fourier transform, analytic k-space update,
// inverse transform) and Sec. 2.5.2 (fill G2 guards from G1, copy the interior
// back).  The real-to-complex and complex-to-real x transforms pack two
// neighbouring real y-lines into one complex line: with z = a + i b,
//   A(k) = (Z(k) + conj Z(-k)) / 2,   B(k) = (Z(k) - conj Z(-k)) / (2 i),
// and the inverse rebuilds Z = A + i B over the full line from the half
// spectra (imaginary parts of the self-conjugate bins dropped).
//
// Every kernel is persistent: a block loads a tile into LDS (through registers,
// in rounds of a few values per thread), transforms it, writes it out and takes
// the next tile.  Blocks are small enough in registers (FP32: at most 128, 96 for
// the z pass and 80 for the single-box y pass, whatever that costs in spills) that
// several share a CU and overlap one another's loads, transforms and barriers.
// All global accesses go through buffer resources with hardware range checks
// (gmem.hpp); an index that is out of range by construction (kOOB) reads zero
// and drops writes.
//
// Each pass body is written against a parameter source: a single box (the
// parameters are the kernel argument) or a batch of boxes of different sizes
// (per-box parameters in device memory, tiles of all boxes numbered one after
// the other).  A batched launch is one persistent grid over the tiles of every
// box (Fig. 1(a) of the paper: many sub-domains, each advanced on its own).

#include "internal.hpp"

namespace psatd {

namespace {

constexpr uint32_t kOOB = 0x3fffffffu;  // element index past the end of every array

template <typename T>
__device__ inline cx<T>* lds_base() {
  extern __shared__ double2 psatd_smem[];
  return reinterpret_cast<cx<T>*>(psatd_smem);
}

// x mod d for 0 <= x < 2^31
__device__ __forceinline__ int fmod_i(int x, const FastDiv& f) { return x - fdiv(x, f) * (int)f.d; }
// x mod d for 0 <= x < 2 d
__device__ __forceinline__ int wrap_once(int x, int d) { return x - (x >= d ? d : 0); }
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// ------------------------------------------------------------------ parameter sources
// A single box's parameters are the kernel's only argument, so they sit at
// offset 0 of the kernel-argument segment.  They are read from there through a
// pointer: binding a reference to the by-value argument makes the compiler keep
// a private (scratch) copy of the whole block, because the transform schedules
// inside it are indexed with run-time stage numbers.
template <typename P>
struct SingleSrc {
  const P* p;
  __device__ __forceinline__ SingleSrc()
      : p((const P*)__builtin_amdgcn_kernarg_segment_ptr()) {}
  __device__ __forceinline__ int ntiles() const { return p->ntiles; }
  __device__ __forceinline__ const P& box(int tile, int& local) const {
    local = tile;
    return *p;
  }
};

template <typename P>
struct BatchSrc {
  BatchArgs<P> a;
  __device__ __forceinline__ int ntiles() const { return a.total; }
  // box b with starts[b] <= tile < starts[b + 1] (binary search on uniform values)
  __device__ __forceinline__ const P& box(int tile, int& local) const {
    int lo = 0, hi = a.nbox;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (a.starts[mid] <= tile)
        lo = mid;
      else
        hi = mid;
    }
    local = tile - a.starts[lo];
    return a.descs[lo];
  }
};

// Cache policy of the x passes' stores: streamed (non-temporal) in FP32, where it made the
// step about 3 % faster; FP64 was slower with it and keeps the default.
template <typename T>
constexpr int kXStore = sizeof(T) == 4 ? kStream : kKeep;

// ------------------------------------------------------------------ P1
// Tiles are ty consecutive y rows of one (field, z) plane, packed as ty/2
// complex lines.  Loads go to LDS in rounds of load_round values per thread;
// overlap comes from several blocks per CU.
template <typename T, typename Src>
__device__ __forceinline__ void xfwd_body(const Src& S) {
  constexpr int kRound = load_round<T>::v;  // element pairs loaded per thread before they go to LDS
  cx<T>* lds = lds_base<T>();
  const int tid = threadIdx.x, nth = blockDim.x;

  for (int tile = blockIdx.x; tile < S.ntiles(); tile += gridDim.x) {
    int lt;
    const XFwdParams<T>& p = S.box(tile, lt);
    const int q = fdiv(lt, p.fd_ytiles);
    const int ybase = (lt - q * p.ytiles) * p.ty;
    const int f = fdiv(q, p.fd_NZ);
    const int z = q - f * p.NZ;
    const int NX = p.NX, NY = p.NY, NXH = p.NXH, ty = p.ty, nc = ty >> 1;
    const int ld = fft_slots(p.fft.sch.n);
    const int nld = nc * NX;
    {
      const rsrc_t src = make_rsrc(p.src[f], p.src_bytes);
      const int zrow = p.gather ? fmod_i(p.z0 + z, p.fd_GZ) * p.GY : z * NY;
      const int rowlen = p.gather ? p.GX : NX;
      // Gather table, after the tile's lines: the wrapped x of every column, then the G1
      // offset of every real row of the tile, so the loads below need no divisions.
      int* tab = reinterpret_cast<int*>(lds + nc * ld);
      if (p.xtab) {
        for (int i = tid; i < NX + ty; i += nth)
          tab[i] = i < NX ? fmod_i(p.x0 + i, p.fd_GX) : (zrow + fmod_i(p.y0 + ybase + (i - NX), p.fd_GY)) * rowlen;
        __syncthreads();
      }
      Walk w;
      w.row = fdiv(tid, p.fd_NX);
      w.col = tid - w.row * NX;
      for (int e0 = 0; e0 < nld; e0 += kRound * nth) {
        T re[kRound], im[kRound];
        Walk w0 = w;
#pragma unroll
        for (int u = 0; u < kRound; ++u) {
          uint32_t ia = kOOB, ib = kOOB;
          if (e0 + tid + u * nth < nld) {
            const int ya = ybase + 2 * w.row;
            int xs = w.col, ra = ya, rb = ya + 1;
            if (p.xtab) {
              const int xt = tab[w.col];
              if (ya < NY) ia = (uint32_t)(tab[NX + 2 * w.row] + xt);
              if (ya + 1 < NY) ib = (uint32_t)(tab[NX + 2 * w.row + 1] + xt);
            } else {
              if (p.gather) {
                xs = fmod_i(p.x0 + w.col, p.fd_GX);
                ra = fmod_i(p.y0 + ya, p.fd_GY);
                rb = fmod_i(p.y0 + ya + 1, p.fd_GY);
              }
              if (ya < NY) ia = (uint32_t)((zrow + ra) * rowlen + xs);
              if (ya + 1 < NY) ib = (uint32_t)((zrow + rb) * rowlen + xs);
            }
          }
          re[u] = gm<T>::ld(src, ia);
          im[u] = gm<T>::ld(src, ib);
          w.next(p.ld_drow, p.ld_dcol, NX);
        }
#pragma unroll
        for (int u = 0; u < kRound; ++u) {
          if (e0 + tid + u * nth < nld) lds[w0.row * ld + lpad(w0.col)] = {re[u], im[u]};
          w0.next(p.ld_drow, p.ld_dcol, NX);
        }
      }
    }
    __syncthreads();
    lds_line_fft<-1, T>(lds, ld, nc, p.fft);

    // Split each complex line c into the half spectra of its two real lines
    // (y = 2c and 2c + 1), written as one pair; y fastest.
    const rsrc_t dst = make_rsrc(p.dst + (i64)f * p.npts, p.dst_bytes);
    const int ny_t = min(ty, NY - ybase);
    const int nwr = NXH * nc;
    Walk v;
    v.row = fdiv(tid, p.fd_nc);
    v.col = tid - v.row * nc;
#pragma unroll 2
    for (int e = tid; e < nwr; e += nth) {
      const int kx = v.row, c = v.col;
      const cx<T> za = lds[c * ld + lpad(kx)];
      const cx<T> zb = cconj(lds[c * ld + lpad(kx == 0 ? 0 : NX - kx)]);
      const cx<T> sum = cadd(za, zb), dif = csub(za, zb);
      const cx<T> va = cscale(sum, T(0.5));
      const cx<T> vb = {T(0.5) * dif.im, T(-0.5) * dif.re};
      const int t = 2 * c;
      const uint32_t o = (uint32_t)((z * NXH + kx) * NY + ybase + t);
      // streamed: layout A is read back by the y pass after all of it has been written
      if (t + 1 < ny_t)
        gm<T>::template stc2<kXStore<T>>(dst, o, va, vb);
      else if (t < ny_t)
        gm<T>::template stc<kXStore<T>>(dst, o, va);
      v.next(p.wr_drow, p.wr_dcol, nc);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ P1 / P5, two-stage lines
// The x passes of a single box for lines of N = RA * RB points with compile-time
// radices (the stage structure of the two-stage y and z kernels), NL complex
// lines (2 NL real rows) per tile.  P1: stage A gathers each butterfly's RA
// points of its two real rows straight from G1 (or the box) into registers,
// stage B leaves the transform in natural order in LDS, and the split into the
// two rows' half spectra is written as before.  P5: the half spectra of two
// rows are rebuilt into a full line in LDS, both stages run from LDS, and the
// rows (real part to one, imaginary part to the other) are written along x from
// the natural-order line: stage B's own outputs are RA points apart, and
// storing them straight from registers would split every wave's stores into
// short runs of several rows.
template <typename T, int RA, int RB, int NL, int NTH>
__device__ __forceinline__ void xfwd_two_stage_body(const XFwdParams<T>& p) {
  constexpr int N = RA * RB, PA = RA | 1, LD = two_stage_slots(RA, RB);
  cx<T>* lds = lds_base<T>();
  int* xoff = reinterpret_cast<int*>(lds + NL * LD);  // source column of each box x (G1 wrap applied)
  // stage B twiddles w^(t k), copied once per launch to LDS as [t - 1][k], after the column table
  Tw<T>* twl = reinterpret_cast<Tw<T>*>(xoff + ((RA * RB + 3) & ~3));
  for (int i = threadIdx.x; i < RA * (RB - 1); i += NTH) {
    const int k = i / (RB - 1), t = i - k * (RB - 1);
    twl[t * RA + k] = p.fft.tw[(RA - 1) + i];
  }
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NTH) xoff[i] = p.gather ? fmod_i(p.x0 + i, p.fd_GX) : i;
  __syncthreads();
  const int NY = p.NY, NXH = p.NXH;
  const int rowlen = p.gather ? p.GX : N;
  for (int tile = blockIdx.x; tile < p.ntiles; tile += gridDim.x) {
    const int q = fdiv(tile, p.fd_ytiles);
    const int ybase = (tile - q * p.ytiles) * (2 * NL);
    const int f = fdiv(q, p.fd_NZ);
    const int z = q - f * p.NZ;
    const int zrow = p.gather ? fmod_i(p.z0 + z, p.fd_GZ) * p.GY : z * NY;
    // stage A: rows a = ybase + 2c, b = a + 1 of line c as one complex line
    {
      const rsrc_t src = make_rsrc(p.src[f], p.src_bytes);
#pragma unroll
      for (int b0 = 0; b0 < NL * RB; b0 += NTH) {
        const int bi = b0 + tid;
        if (b0 + NTH <= NL * RB || bi < NL * RB) {
          const int c = bi / RB, j = bi - c * RB;
          const int ya = ybase + 2 * c;
          int ra = ya, rb = ya + 1;
          if (p.gather) {
            ra = fmod_i(p.y0 + ya, p.fd_GY);
            rb = fmod_i(p.y0 + ya + 1, p.fd_GY);
          }
          const uint32_t oa = ya < NY ? (uint32_t)((zrow + ra) * rowlen) : kOOB;
          const uint32_t ob = ya + 1 < NY ? (uint32_t)((zrow + rb) * rowlen) : kOOB;
          cx<T> v[RA];
#pragma unroll
          for (int t = 0; t < RA; ++t) {
            const int xs = xoff[j + RB * t];
            v[t] = {gm<T>::ld(src, oa + (uint32_t)xs), gm<T>::ld(src, ob + (uint32_t)xs)};
          }
          dft<RA, -1, T>::run(v);
          cx<T>* y = lds + c * LD + j * PA;
#pragma unroll
          for (int t = 0; t < RA; ++t) y[t] = v[t];
        }
      }
    }
    __syncthreads();
    // stage B: rows -> twiddles -> DFT -> natural order (in place, after all reads)
    {
      constexpr int NBR = (NL * RA + NTH - 1) / NTH;
      cx<T> v[NBR][RB];
#pragma unroll
      for (int u = 0; u < NBR; ++u) {
        const int bi = u * NTH + tid;
        if (bi < NL * RA) {
          const int c = bi / RA, k = bi - c * RA;
          const cx<T>* y = lds + c * LD + k;
#pragma unroll
          for (int t = 0; t < RB; ++t) v[u][t] = y[t * PA];
          if (k > 0) {
#pragma unroll
            for (int t = 1; t < RB; ++t) v[u][t] = twmul<-1>(v[u][t], twl[(t - 1) * RA + k]);
          }
          dft<RB, -1, T>::run(v[u]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NBR; ++u) {
        const int bi = u * NTH + tid;
        if (bi < NL * RA) {
          const int c = bi / RA, k = bi - c * RA;
          cx<T>* zl = lds + c * LD + k;
#pragma unroll
          for (int t = 0; t < RB; ++t) zl[t * RA] = v[u][t];
        }
      }
    }
    __syncthreads();
    // split each complex line into the half spectra of its two real rows, written as pairs
    const rsrc_t dst = make_rsrc(p.dst + (i64)f * p.npts, p.dst_bytes);
    const int ny_t = min(2 * NL, NY - ybase);
    for (int e = tid; e < NXH * NL; e += NTH) {
      const int kx = e / NL, c = e - kx * NL;
      const cx<T> za = lds[c * LD + kx];
      const cx<T> zb = cconj(lds[c * LD + (kx == 0 ? 0 : N - kx)]);
      const cx<T> sum = cadd(za, zb), dif = csub(za, zb);
      const cx<T> va = cscale(sum, T(0.5));
      const cx<T> vb = {T(0.5) * dif.im, T(-0.5) * dif.re};
      const int t = 2 * c;
      const uint32_t o = (uint32_t)((z * NXH + kx) * NY + ybase + t);
      // streamed: layout A is read back by the y pass after all of it has been written
      if (t + 1 < ny_t)
        gm<T>::template stc2<kXStore<T>>(dst, o, va, vb);
      else if (t < ny_t)
        gm<T>::template stc<kXStore<T>>(dst, o, va);
    }
    __syncthreads();
  }
}

template <typename T, int RA, int RB, int NL, int NTH>
__device__ __forceinline__ void xinv_two_stage_body(const XInvParams<T>& p) {
  constexpr int N = RA * RB, PA = RA | 1, LD = two_stage_slots(RA, RB);
  cx<T>* lds = lds_base<T>();
  // stage B twiddles w^(t k), copied once per launch to LDS as [t - 1][k]
  Tw<T>* twl = reinterpret_cast<Tw<T>*>(lds + NL * LD);
  for (int i = threadIdx.x; i < RA * (RB - 1); i += NTH) {
    const int k = i / (RB - 1), t = i - k * (RB - 1);
    twl[t * RA + k] = p.fft.tw[(RA - 1) + i];
  }
  const int tid = threadIdx.x;
  const int NY = p.NY, NXH = p.NXH;
  for (int tile = blockIdx.x; tile < p.ntiles; tile += gridDim.x) {
    const int q = fdiv(tile, p.fd_ytiles);
    const int ybase = p.y_lo + (tile - q * p.ytiles) * (2 * NL);
    const int f = fdiv(q, p.fd_nz);
    const int z = p.z_lo + (q - f * (p.z_hi - p.z_lo));
    // rebuild Z = A + i B over the full line from the half spectra of rows 2c, 2c + 1;
    // every load of the tile is issued before the first LDS write
    {
      constexpr int NH = N / 2 + 1;
      constexpr int NR = (NH * NL + NTH - 1) / NTH;
      const rsrc_t src = make_rsrc(p.src + (i64)f * p.npts, p.src_bytes);
      const int sbase = z * NXH * NY;
      cx<T> xa[NR], xb[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int e = r * NTH + tid;
        const int kx = e / NL, c = e - kx * NL;
        const int ya = ybase + 2 * c;
        const bool ok = e < NH * NL;
        xa[r] = gm<T>::ldc(src, ok && ya < p.y_hi ? (uint32_t)(sbase + kx * NY + ya) : kOOB);
        xb[r] = gm<T>::ldc(src, ok && ya + 1 < p.y_hi ? (uint32_t)(sbase + kx * NY + ya + 1) : kOOB);
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int e = r * NTH + tid;
        if (e >= NH * NL) break;
        const int kx = e / NL, c = e - kx * NL;
        cx<T> x = xa[r], y = xb[r];
        const bool selfconj = (kx == 0) || (2 * kx == N);
        if (selfconj) {
          x.im = T(0);
          y.im = T(0);
        }
        lds[c * LD + kx] = {x.re - y.im, x.im + y.re};
        if (!selfconj) lds[c * LD + (N - kx)] = {x.re + y.im, y.re - x.im};
      }
    }
    __syncthreads();
    // stage A from the natural-order line, in place after all reads
    {
      constexpr int NAR = (NL * RB + NTH - 1) / NTH;
      cx<T> v[NAR][RA];
#pragma unroll
      for (int u = 0; u < NAR; ++u) {
        const int bi = u * NTH + tid;
        if (bi < NL * RB) {
          const int c = bi / RB, j = bi - c * RB;
          const cx<T>* x = lds + c * LD + j;
#pragma unroll
          for (int t = 0; t < RA; ++t) v[u][t] = x[RB * t];
          dft<RA, 1, T>::run(v[u]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NAR; ++u) {
        const int bi = u * NTH + tid;
        if (bi < NL * RB) {
          const int c = bi / RB, j = bi - c * RB;
          cx<T>* y = lds + c * LD + j * PA;
#pragma unroll
          for (int t = 0; t < RA; ++t) y[t] = v[u][t];
        }
      }
    }
    __syncthreads();
    // stage B: rows -> twiddles -> DFT -> natural order (in place, after all reads)
    {
      constexpr int NBR = (NL * RA + NTH - 1) / NTH;
      cx<T> v[NBR][RB];
#pragma unroll
      for (int u = 0; u < NBR; ++u) {
        const int bi = u * NTH + tid;
        if (bi < NL * RA) {
          const int c = bi / RA, k = bi - c * RA;
          const cx<T>* y = lds + c * LD + k;
#pragma unroll
          for (int t = 0; t < RB; ++t) v[u][t] = y[t * PA];
          if (k > 0) {
#pragma unroll
            for (int t = 1; t < RB; ++t) v[u][t] = twmul<1>(v[u][t], twl[(t - 1) * RA + k]);
          }
          dft<RB, 1, T>::run(v[u]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NBR; ++u) {
        const int bi = u * NTH + tid;
        if (bi < NL * RA) {
          const int c = bi / RA, k = bi - c * RA;
          cx<T>* zl = lds + c * LD + k;
#pragma unroll
          for (int t = 0; t < RB; ++t) zl[t * RA] = v[u][t];
        }
      }
    }
    __syncthreads();
    // the two real rows of each line (box, or interior of G1), written along x so that
    // a wave's stores cover whole rows
    {
      const rsrc_t dst = make_rsrc(p.dst[f], p.dst_bytes);
      const int zrow = p.scatter ? fmod_i(p.oz + z - p.gz, p.fd_GZ) * p.GY : z * NY;
      const int rowlen = p.scatter ? p.GX : N;
      for (int e = tid; e < NL * N; e += NTH) {
        const int c = e / N, n = e - c * N;
        const cx<T> val = lds[c * LD + n];
        const int ya = ybase + 2 * c;
        uint32_t ia = kOOB, ib = kOOB;
        if (!p.scatter) {
          if (ya < p.y_hi) ia = (uint32_t)((zrow + ya) * rowlen + n);
          if (ya + 1 < p.y_hi) ib = (uint32_t)((zrow + ya + 1) * rowlen + n);
        } else if (n >= p.gx && n < p.gx + p.nx) {
          // the interior is no larger than the grid and its origin lies in it: one wrap at most
          const int xg = wrap_once(p.ox + n - p.gx, p.GX);
          const int ra = wrap_once(p.oy + ya - p.gy, p.GY);
          if (ya < p.y_hi) ia = (uint32_t)((zrow + ra) * rowlen + xg);
          if (ya + 1 < p.y_hi) ib = (uint32_t)((zrow + wrap_once(ra + 1, p.GY)) * rowlen + xg);
        }
        // streamed: G1 is read back by the next step's fill
        gm<T>::template st<kXStore<T>>(dst, ia, val.re);
        gm<T>::template st<kXStore<T>>(dst, ib, val.im);
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ P2 / P4
// Tiles are y-lines (about 5k elements); loads go to LDS in rounds of
// load_round values per thread, and several blocks per CU overlap each other.
template <int S_, typename T, typename Src>
__device__ __forceinline__ void ypass_body(const Src& S) {
  constexpr int kRound = load_round<T>::v;
  cx<T>* lds = lds_base<T>();
  const int tid = threadIdx.x, nth = blockDim.x;

  struct Tile {
    int f, o, u0, nlt;
    FastDiv fnl;
  };
  auto decode = [&](const YPassParams<T>& p, int lt) {
    Tile t;
    const int q = fdiv(lt, p.fd_utiles);
    const int ut = lt - q * p.utiles;
    t.f = fdiv(q, p.fd_nouter);
    t.o = q - t.f * p.nouter;
    t.u0 = p.u_lo + ut * p.nl;
    const bool last = (ut == p.utiles - 1);
    t.nlt = last ? p.nl_last : p.nl;
    t.fnl = last ? p.fd_nl_last : p.fd_nl;
    return t;
  };
  // walk over a tile's input elements in the input's preferred order:
  // positions fastest when lines are contiguous, line index fastest otherwise
  auto start_in = [&](const YPassParams<T>& p, const Tile& t, Walk& w, int& dr, int& dc, int& ncol) {
    if (p.ps_in == 1) {
      w.row = fdiv(tid, p.fd_n);
      w.col = tid - w.row * p.n;
      dr = fdiv(nth, p.fd_n);
      dc = nth - dr * p.n;
      ncol = p.n;
    } else {
      w.row = fdiv(tid, t.fnl);
      w.col = tid - w.row * t.nlt;
      dr = fdiv(nth, t.fnl);
      dc = nth - dr * t.nlt;
      ncol = t.nlt;
    }
  };
  for (int tile = blockIdx.x; tile < S.ntiles(); tile += gridDim.x) {
    int lt;
    const YPassParams<T>& p = S.box(tile, lt);
    const Tile t = decode(p, lt);
    const int ld = fft_slots(p.fft.sch.n);
    {
      const rsrc_t in = make_rsrc(p.in + (i64)t.f * p.fs_in, p.in_bytes);
      const int base = t.o * p.os_in + t.u0 * p.ls_in;
      const int tot = t.nlt * p.n;
      Walk w;
      int dr, dc, ncol;
      start_in(p, t, w, dr, dc, ncol);
      for (int e0 = 0; e0 < tot; e0 += kRound * nth) {
        cx<T> r[kRound];
        Walk w0 = w;
#pragma unroll
        for (int u = 0; u < kRound; ++u) {
          uint32_t idx = kOOB;
          if (e0 + tid + u * nth < tot) {
            const int li = (p.ps_in == 1) ? w.row : w.col;
            const int q = (p.ps_in == 1) ? w.col : w.row;
            idx = (uint32_t)(base + li * p.ls_in + q * p.ps_in);
          }
          r[u] = gm<T>::ldc(in, idx);
          w.next(dr, dc, ncol);
        }
#pragma unroll
        for (int u = 0; u < kRound; ++u) {
          if (e0 + tid + u * nth < tot) {
            const int li = (p.ps_in == 1) ? w0.row : w0.col;
            const int q = (p.ps_in == 1) ? w0.col : w0.row;
            lds[li * ld + lpad(q)] = r[u];
          }
          w0.next(dr, dc, ncol);
        }
      }
    }
    __syncthreads();
    lds_line_fft<S_, T>(lds, ld, t.nlt, p.fft);

    const rsrc_t out = make_rsrc(p.out + (i64)t.f * p.fs_out, p.out_bytes);
    const int obase = t.o * p.os_out + t.u0 * p.ls_out;
    const int np = p.p_hi - p.p_lo;
    const int tot = t.nlt * np;
    Walk w;
    int dr, dc, ncol;
    if (p.ps_out == 1) {
      w.row = fdiv(tid, p.fd_np);
      w.col = tid - w.row * np;
      dr = fdiv(nth, p.fd_np);
      dc = nth - dr * np;
      ncol = np;
    } else {
      w.row = fdiv(tid, t.fnl);
      w.col = tid - w.row * t.nlt;
      dr = fdiv(nth, t.fnl);
      dc = nth - dr * t.nlt;
      ncol = t.nlt;
    }
#pragma unroll 4
    for (int e = tid; e < tot; e += nth) {
      const int li = (p.ps_out == 1) ? w.row : w.col;
      const int q = p.p_lo + ((p.ps_out == 1) ? w.col : w.row);
      gm<T>::stc(out, (uint32_t)(obase + li * p.ls_out + q * p.ps_out), lds[li * ld + lpad(q)]);
      w.next(dr, dc, ncol);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ P2 / P4, two-stage lines
// The y passes for lines of N = RA * RB points with compile-time radices and
// tiles of NL lines (the stage structure of the two-stage z kernel below):
// stage A reads each butterfly's RA inputs straight from global memory into
// registers and leaves its outputs in padded LDS rows; stage B reads columns
// of those rows, applies the twiddles and writes its RB outputs straight to
// global memory.  Lanes walk the contiguous direction of each side: along the
// line where positions are contiguous (stride 1), across the tile's lines
// where lines are (P2 writes, P4 reads consecutive z).  The strided offsets
// of a butterfly's points are scalar (the same for every lane), so no lane
// computes a per-point address.  P2 (S_ = -1) reads lines with contiguous
// positions and writes consecutive lines contiguously; P4 (S_ = +1) the reverse.
template <int RA, int RB, int NL>
struct TwoStageY {
  static constexpr int N = RA * RB;
  static constexpr int PA = RA | 1;
  static constexpr int LD = (RB * PA) | 1;
  static constexpr int NA = NL * RB;  // stage A butterflies per tile
  static constexpr int NB = NL * RA;  // stage B butterflies per tile
};

template <int S_, typename T, int RA, int RB, int NL, int NTH, typename Src>
__device__ __forceinline__ void ypass_two_stage_body(const Src& S) {
  using G = TwoStageY<RA, RB, NL>;
  constexpr int PA = G::PA, LD = G::LD;
  cx<T>* lds = lds_base<T>();
  const int tid = threadIdx.x;
  // stage B twiddles w^(t k), copied once per launch to LDS as [t - 1][k]
  Tw<T>* twl = reinterpret_cast<Tw<T>*>(lds + NL * LD);
  {
    int lt0;
    const YPassParams<T>& p0 = S.box(blockIdx.x, lt0);
    for (int i = tid; i < RA * (RB - 1); i += NTH) {
      const int k = i / (RB - 1), t = i - k * (RB - 1);
      twl[t * RA + k] = p0.fft.tw[(RA - 1) + i];
    }
    __syncthreads();
  }
  for (int tile = blockIdx.x; tile < S.ntiles(); tile += gridDim.x) {
    int lt;
    const YPassParams<T>& p = S.box(tile, lt);
    const int q = fdiv(lt, p.fd_utiles);
    const int ut = lt - q * p.utiles;
    const int f = fdiv(q, p.fd_nouter);
    const int o = q - f * p.nouter;
    const int u0 = p.u_lo + ut * NL;
    const int nlt = min(NL, p.u_hi - u0);
    // stage A: global -> registers -> DFT -> padded rows
    {
      const rsrc_t in = make_rsrc(p.in + (i64)f * p.fs_in, p.in_bytes);
      const uint32_t sstep = (uint32_t)(RB * p.ps_in * (int)sizeof(cx<T>));  // bytes between a butterfly's points
#pragma unroll
      for (int b0 = 0; b0 < G::NA; b0 += NTH) {
        const int b = b0 + tid;
        if (b0 + NTH <= G::NA || b < G::NA) {
          const int line = S_ < 0 ? b / RB : b % NL;
          const int j = S_ < 0 ? b - line * RB : b / NL;
          const bool ok = line < nlt;
          const uint32_t base = ok ? (uint32_t)(o * p.os_in + (u0 + line) * p.ls_in + j * p.ps_in) : kOOB;
          cx<T> v[RA];
#pragma unroll
          for (int t = 0; t < RA; ++t) v[t] = gm<T>::ldc_s(in, base, (uint32_t)t * sstep);
          dft<RA, S_, T>::run(v);
          cx<T>* y = lds + line * LD + j * PA;
#pragma unroll
          for (int t = 0; t < RA; ++t) y[t] = v[t];
        }
      }
    }
    __syncthreads();
    // stage B: padded rows -> twiddles -> DFT -> global (positions [p_lo, p_hi))
    {
      const rsrc_t out = make_rsrc(p.out + (i64)f * p.fs_out, p.out_bytes);
      const uint32_t sstep = (uint32_t)(RA * p.ps_out * (int)sizeof(cx<T>));
#pragma unroll
      for (int b0 = 0; b0 < G::NB; b0 += NTH) {
        const int b = b0 + tid;
        if (b0 + NTH <= G::NB || b < G::NB) {
          const int line = S_ > 0 ? b / RA : b % NL;
          const int k = S_ > 0 ? b - line * RA : b / NL;
          const cx<T>* y = lds + line * LD + k;
          cx<T> v[RB];
#pragma unroll
          for (int t = 0; t < RB; ++t) v[t] = y[t * PA];
          if (k > 0) {
#pragma unroll
            for (int t = 1; t < RB; ++t) v[t] = twmul<S_>(v[t], twl[(t - 1) * RA + k]);
          }
          dft<RB, S_, T>::run(v);
          const bool ok = line < nlt;
          const uint32_t base = (uint32_t)(o * p.os_out + (u0 + line) * p.ls_out + k * p.ps_out);
#pragma unroll
          for (int t = 0; t < RB; ++t) {
            const int pos = k + RA * t;
            gm<T>::stc_s(out, (ok && pos >= p.p_lo && pos < p.p_hi) ? base : kOOB, (uint32_t)t * sstep, v[t]);
          }
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ P3
// Push (Sec. 1.1; J constant over the step, rho at both ends):
//   E' = C E + i c^2 S1 (K x B) - (S1/eps0) J + i (c^2/eps0) K (X3 rho_old - X2 rho_new)
//   B' = C B - i S1 (K x E) + i (X1/eps0) (K x J)
// A tile is ncol consecutive (kx, ky) columns (one for long lines, several for
// short ones): their 11 z-lines each are loaded into LDS, transformed, pushed
// point by point, and the 6 lines of E and B per column transformed back and
// stored over the interior z range.  LDS line f * ncol + c holds field f of
// the tile's column c, so the E and B lines of all columns come first and the
// inverse transform runs over one contiguous block of 6 ncol lines (the last
// tile of a box may have fewer columns: its missing lines hold zeros).  This pass
// does not hold the next tile in registers: the transforms leave no room for
// it, and small blocks with a 96-register cap (FP32, five per CU) let several
// tiles per CU overlap each other's loads and barriers instead.
// The push at one k-space point: column col, z index kz, its field-0 value at LDS
// slot s and field f at s + f * fs; k_x, k_y of the column given.
// Staggered grid: the same update with the complex symbols kappa = k_s exp(i k d / 2)
// (kp, from nodes to the half points above) and their conjugates (back down):
//   E' = C E + i c^2 S1 (kappa^* x B) - (S1/eps0) J + i (c^2/eps0) kappa (X3 rho_old - X2 rho_new)
//   B' = C B - i S1 (kappa x E) + i (X1/eps0) (kappa x J)
// (E and J sit half a cell up along their own axis, B along the other two, rho on
// the nodes; C, S1, X1..X3 are functions of |k_s|).
template <typename T>
__device__ __forceinline__ void push_point_staggered(const ZPushParams<T>& p, cx<T>* lds, int fs, int s, int kz,
                                                     cx<T> kx, cx<T> ky, const T* cc) {
  const T c2 = p.c2, ie = p.inv_eps0;
  const T C = cc[0], S1 = cc[1], X1 = cc[2], X2 = cc[3], X3 = cc[4];
  const cx<T> kz_ = p.kzc[kz];
  const cx<T> kxm = cconj(kx), kym = cconj(ky), kzm = cconj(kz_);
  const cx<T> ex = lds[0 * fs + s], ey = lds[1 * fs + s], ez = lds[2 * fs + s];
  const cx<T> bx = lds[3 * fs + s], by = lds[4 * fs + s], bz = lds[5 * fs + s];
  const cx<T> jx = lds[6 * fs + s], jy = lds[7 * fs + s], jz = lds[8 * fs + s];
  const cx<T> ro = lds[9 * fs + s], rn = lds[10 * fs + s];
  // kappa^* x B, kappa x E, kappa x J
  const cx<T> kbx = csub(cmul(kym, bz), cmul(kzm, by));
  const cx<T> kby = csub(cmul(kzm, bx), cmul(kxm, bz));
  const cx<T> kbz = csub(cmul(kxm, by), cmul(kym, bx));
  const cx<T> kex = csub(cmul(ky, ez), cmul(kz_, ey));
  const cx<T> key = csub(cmul(kz_, ex), cmul(kx, ez));
  const cx<T> kez = csub(cmul(kx, ey), cmul(ky, ex));
  const cx<T> kjx = csub(cmul(ky, jz), cmul(kz_, jy));
  const cx<T> kjy = csub(cmul(kz_, jx), cmul(kx, jz));
  const cx<T> kjz = csub(cmul(kx, jy), cmul(ky, jx));
  const cx<T> rr = csub(cscale(ro, X3), cscale(rn, X2));
  const T a = c2 * S1, g = c2 * ie, sj = S1 * ie, xj = X1 * ie;
  const cx<T> ux = cadd(cscale(kbx, a), cscale(cmul(kx, rr), g));
  const cx<T> uy = cadd(cscale(kby, a), cscale(cmul(ky, rr), g));
  const cx<T> uz = cadd(cscale(kbz, a), cscale(cmul(kz_, rr), g));
  lds[0 * fs + s] = {C * ex.re - sj * jx.re - ux.im, C * ex.im - sj * jx.im + ux.re};
  lds[1 * fs + s] = {C * ey.re - sj * jy.re - uy.im, C * ey.im - sj * jy.im + uy.re};
  lds[2 * fs + s] = {C * ez.re - sj * jz.re - uz.im, C * ez.im - sj * jz.im + uz.re};
  const cx<T> wx = csub(cscale(kjx, xj), cscale(kex, S1));
  const cx<T> wy = csub(cscale(kjy, xj), cscale(key, S1));
  const cx<T> wz = csub(cscale(kjz, xj), cscale(kez, S1));
  lds[3 * fs + s] = {C * bx.re - wx.im, C * bx.im + wx.re};
  lds[4 * fs + s] = {C * by.re - wy.im, C * by.im + wy.re};
  lds[5 * fs + s] = {C * bz.re - wz.im, C * bz.im + wz.re};
}

template <typename T>
__device__ __forceinline__ void push_point_c(const ZPushParams<T>& p, cx<T>* lds, int fs, int s, int kz,
                                             int kxi, int kyi, const T* cc);
template <typename T>
__device__ __forceinline__ void push_point_pml(const ZPushParams<T>& p, cx<T>* lds, int fs, int s, int kz,
                                               int kxi, int kyi, const T* cc);
template <typename T, bool PML = false>
__device__ __forceinline__ void push_point(const ZPushParams<T>& p, cx<T>* lds, int fs, int s, int col, int kz,
                                           int kxi, int kyi) {
  const uint32_t idx = (uint32_t)(col * p.NZ + kz);
  T cc[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) cc[k] = gm<T>::ld(make_rsrc(p.coef + (i64)k * p.npts, p.coef_bytes), idx);
  if constexpr (PML)
    push_point_pml(p, lds, fs, s, kz, kxi, kyi, cc);
  else
    push_point_c(p, lds, fs, s, kz, kxi, kyi, cc);
}
template <typename T>
__device__ __forceinline__ void push_point_c(const ZPushParams<T>& p, cx<T>* lds, int fs, int s, int kz,
                                             int kxi, int kyi, const T* cc) {
  const T c2 = p.c2, ie = p.inv_eps0;
  if (p.stag) {
    push_point_staggered(p, lds, fs, s, kz, p.kxc[kxi], p.kyc[kyi], cc);
    return;
  }
  const T kx = p.kx[kxi], ky = p.ky[kyi];
  const T C = cc[0], S1 = cc[1], X1 = cc[2], X2 = cc[3], X3 = cc[4];
  const T kzz = p.kz[kz];
  const cx<T> ex = lds[0 * fs + s], ey = lds[1 * fs + s], ez = lds[2 * fs + s];
  const cx<T> bx = lds[3 * fs + s], by = lds[4 * fs + s], bz = lds[5 * fs + s];
  const cx<T> jx = lds[6 * fs + s], jy = lds[7 * fs + s], jz = lds[8 * fs + s];
  const cx<T> ro = lds[9 * fs + s], rn = lds[10 * fs + s];
  // K x B, K x E, K x J (K real)
  const cx<T> kbx = csub(cscale(bz, ky), cscale(by, kzz));
  const cx<T> kby = csub(cscale(bx, kzz), cscale(bz, kx));
  const cx<T> kbz = csub(cscale(by, kx), cscale(bx, ky));
  const cx<T> kex = csub(cscale(ez, ky), cscale(ey, kzz));
  const cx<T> key = csub(cscale(ex, kzz), cscale(ez, kx));
  const cx<T> kez = csub(cscale(ey, kx), cscale(ex, ky));
  const cx<T> kjx = csub(cscale(jz, ky), cscale(jy, kzz));
  const cx<T> kjy = csub(cscale(jx, kzz), cscale(jz, kx));
  const cx<T> kjz = csub(cscale(jy, kx), cscale(jx, ky));
  const cx<T> rr = csub(cscale(ro, X3), cscale(rn, X2));
  const T a = c2 * S1;   // multiplies K x B
  const T g = c2 * ie;   // multiplies K r
  const T sj = S1 * ie;  // multiplies J
  const T xj = X1 * ie;  // multiplies K x J
  // E' = C E - sj J + i (a K x B + g K r)
  const cx<T> ux = cadd(cscale(kbx, a), cscale(rr, g * kx));
  const cx<T> uy = cadd(cscale(kby, a), cscale(rr, g * ky));
  const cx<T> uz = cadd(cscale(kbz, a), cscale(rr, g * kzz));
  lds[0 * fs + s] = {C * ex.re - sj * jx.re - ux.im, C * ex.im - sj * jx.im + ux.re};
  lds[1 * fs + s] = {C * ey.re - sj * jy.re - uy.im, C * ey.im - sj * jy.im + uy.re};
  lds[2 * fs + s] = {C * ez.re - sj * jz.re - uz.im, C * ez.im - sj * jz.im + uz.re};
  // B' = C B + i (xj K x J - S1 K x E)
  const cx<T> wx = csub(cscale(kjx, xj), cscale(kex, S1));
  const cx<T> wy = csub(cscale(kjy, xj), cscale(key, S1));
  const cx<T> wz = csub(cscale(kjz, xj), cscale(kez, S1));
  lds[3 * fs + s] = {C * bx.re - wx.im, C * bx.im + wx.re};
  lds[4 * fs + s] = {C * by.re - wy.im, C * by.im + wy.re};
  lds[5 * fs + s] = {C * bz.re - wz.im, C * bz.im + wz.re};
}

// Two-step PML (Sec. 2.6): the twelve split parts of E and B (component a split into set
// A, driven by the derivative along axis a+1, and set B, along a+2) advance over the step
// by the integral of their own right-hand side along the exact evolution of the full
// fields, with the sources constant.  Set B of E_a gains -i c^2 K_{a+2} IB_{a+1}, set B of
// B_a gains +i K_{a+2} IE_{a+1}, where
//   IB = S1 B_T + dt B_L - i X1 (K x E) + i (dt X2/eps0) (K x J),
//   IE = S1 E_T + dt E_L + i c^2 X1 (K x B) - (X1/eps0) J_T - (dt^2/(2 eps0)) J_L
// are the integrals of B(t) and E(t) over the step (T, L: parts transverse and parallel
// to K); set A takes the rest of the increment of the ordinary push, so the two sets
// always add up to it.  Writes the increments (scaled by 1/N like the tables) of set A
// to slots 0..5 and of set B to slots 6..11 (in the split-part order E_xz E_yx E_zy
// B_xz B_yx B_zy); the sources in slots 6..10 are read first.  Collocated grid.
template <typename T>
__device__ __forceinline__ void push_point_pml(const ZPushParams<T>& p, cx<T>* lds, int fs, int s, int kz,
                                               int kxi, int kyi, const T* cc) {
  const T c2 = p.c2, ie = p.inv_eps0, invn = p.inv_n, dt = p.dt;
  const T K[3] = {p.kx[kxi], p.ky[kyi], p.kz[kz]};
  const T C = cc[0], S1 = cc[1], X1 = cc[2], X2 = cc[3], X3 = cc[4];
  cx<T> E[3], B[3], J[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    E[a] = lds[a * fs + s];
    B[a] = lds[(3 + a) * fs + s];
    J[a] = lds[(6 + a) * fs + s];
  }
  const cx<T> ro = lds[9 * fs + s], rn = lds[10 * fs + s];
  const T k2 = K[0] * K[0] + K[1] * K[1] + K[2] * K[2];
  const T ik2 = k2 > T(0) ? T(1) / k2 : T(0);
  auto dot = [&](const cx<T>* v) {
    return cadd(cadd(cscale(v[0], K[0]), cscale(v[1], K[1])), cscale(v[2], K[2]));
  };
  auto cross = [&](const cx<T>* v, int a) {  // (K x v)_a
    const int b = a == 2 ? 0 : a + 1, c = a == 0 ? 2 : a - 1;
    return csub(cscale(v[c], K[b]), cscale(v[b], K[c]));
  };
  const cx<T> kE = cscale(dot(E), ik2), kB = cscale(dot(B), ik2), kJ = cscale(dot(J), ik2);
  const cx<T> rr = csub(cscale(ro, X3), cscale(rn, X2));
  cx<T> IB[3], IE[3], dE[3], dB[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cx<T> kxe = cross(E, a), kxb = cross(B, a), kxj = cross(J, a);
    const cx<T> EL = cscale(kE, K[a]), BL = cscale(kB, K[a]), JL = cscale(kJ, K[a]);
    // IB_a = S1 (B - B_L) + dt/N B_L + (X1 K x E + dt X2/eps0 K x J) * (-i, +i)
    const cx<T> ib_r = cadd(cscale(csub(B[a], BL), S1), cscale(BL, dt * invn));
    const cx<T> ib_i = csub(cscale(kxj, dt * X2 * ie), cscale(kxe, X1));  // times i
    IB[a] = {ib_r.re - ib_i.im, ib_r.im + ib_i.re};
    const cx<T> ie_r = csub(cadd(cscale(csub(E[a], EL), S1), cscale(EL, dt * invn)),
                            cadd(cscale(csub(J[a], JL), X1 * ie), cscale(JL, T(0.5) * dt * dt * invn * ie)));
    const cx<T> ie_i = cscale(kxb, c2 * X1);  // times i
    IE[a] = {ie_r.re - ie_i.im, ie_r.im + ie_i.re};
    // ordinary push (tables scaled by 1/N) minus E/N: the whole increment
    const cx<T> ux = cadd(cscale(kxb, c2 * S1), cscale(rr, c2 * ie * K[a]));
    dE[a] = {C * E[a].re - S1 * ie * J[a].re - ux.im - invn * E[a].re,
             C * E[a].im - S1 * ie * J[a].im + ux.re - invn * E[a].im};
    const cx<T> w = csub(cscale(kxj, X1 * ie), cscale(kxe, S1));
    dB[a] = {C * B[a].re - w.im - invn * B[a].re, C * B[a].im + w.re - invn * B[a].im};
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int b = a == 2 ? 0 : a + 1, c = a == 0 ? 2 : a - 1;  // a+1, a+2
    // set B: -i c^2 K_c IB_b and +i K_c IE_b
    const cx<T> eb = {c2 * K[c] * IB[b].im, -c2 * K[c] * IB[b].re};
    const cx<T> bb = {-K[c] * IE[b].im, K[c] * IE[b].re};
    lds[a * fs + s] = csub(dE[a], eb);
    lds[(3 + a) * fs + s] = csub(dB[a], bb);
    lds[(6 + a) * fs + s] = eb;
    lds[(9 + a) * fs + s] = bb;
  }
}

// MULTI = false compiles the single-column case (ncol == 1) without the column bookkeeping.
// PML selects the split-field increments of push_point_pml instead of the ordinary push:
// twelve output lines per column (both split sets) instead of six.
template <typename T, bool MULTI, typename Src, bool PML = false>
__device__ __forceinline__ void zpush_body(const Src& S) {
  constexpr int kRound = 16;  // line chunks of 64 points loaded per thread before they go to LDS
  cx<T>* lds = lds_base<T>();
  const int tid = threadIdx.x, nth = blockDim.x;
  const int lane = tid & 63;
  const int wave = uniform(tid >> 6);
  const int nwaves = nth >> 6;
  for (int tile = blockIdx.x; tile < S.ntiles(); tile += gridDim.x) {
    int lt;
    const ZPushParams<T>& p = S.box(tile, lt);
    const int NZ = p.NZ;
    const int ld = fft_slots(p.fft.sch.n);
    const int col0 = lt * p.ncol;
    const int ncol = MULTI ? p.ncol : 1;
    const int nct = MULTI ? min(ncol, p.NXH * p.NY - col0) : 1;  // columns present in this tile
    const int nlines = 11 * ncol;
    const int per_line = (NZ + 63) >> 6;
    const int items = ((nlines - wave + nwaves - 1) / nwaves) * per_line;  // (line, chunk) pairs of this wave
    for (int q0 = 0; q0 < items; q0 += kRound) {
      cx<T> r[kRound];
#pragma unroll
      for (int u = 0; u < kRound; ++u) {
        const int q = q0 + u;
        const int sl = q / per_line, i = q - sl * per_line;
        const int l = wave + sl * nwaves;  // LDS line: field l / ncol, column l % ncol
        const int f = MULTI ? fdiv(l, p.fd_ncol) : l, c = MULTI ? l - f * ncol : 0;
        const int z = lane + 64 * i;
        const bool ok = q < items && z < NZ && (!MULTI || c < nct);
        const rsrc_t rb = make_rsrc(p.b + (i64)(ok ? f : 0) * p.npts, p.field_bytes);
        r[u] = gm<T>::ldc(rb, ok ? (uint32_t)((col0 + c) * NZ + z) : kOOB);
      }
#pragma unroll
      for (int u = 0; u < kRound; ++u) {
        const int q = q0 + u;
        const int sl = q / per_line, i = q - sl * per_line;
        const int z = lane + 64 * i;
        if (q < items && z < NZ) lds[(wave + sl * nwaves) * ld + lpad(z)] = r[u];
      }
    }
    __syncthreads();
    // lines are independent: transform them in groups that fit the block's butterfly budget
    if (p.zgroup >= nlines)
      lds_line_fft<-1, T>(lds, ld, nlines, p.fft);
    else
      for (int l0 = 0; l0 < nlines; l0 += p.zgroup)
        lds_line_fft<-1, T>(lds + l0 * ld, ld, min(p.zgroup, nlines - l0), p.fft);

    const int fs = ncol * ld;  // LDS distance between the lines of consecutive fields
    if (!MULTI || 2 * NZ > nth) {
      // long lines: one column at a time, its k_x and k_y uniform
      for (int c = 0; c < nct; ++c) {
        const int col = col0 + c;
        const int kxi = fdiv(col, p.fd_NY);
        const int kyi = col - kxi * p.NY;
        for (int kz = tid; kz < NZ; kz += nth) push_point<T, PML>(p, lds, fs, c * ld + lpad(kz), col, kz, kxi, kyi);
      }
    } else {
      // short lines: (column, k_z) pairs spread over the block
      for (int e = tid; e < nct * NZ; e += nth) {
        const int c = fdiv(e, p.fd_NZ);
        const int kz = e - c * NZ;
        const int col = col0 + c;
        const int kxi = fdiv(col, p.fd_NY);
        const int kyi = col - kxi * p.NY;
        push_point<T, PML>(p, lds, fs, c * ld + lpad(kz), col, kz, kxi, kyi);
      }
    }
    __syncthreads();
    constexpr int kOut = PML ? 12 : 6;  // output lines per column
    if (p.zgroup >= kOut * ncol)
      lds_line_fft<1, T>(lds, ld, kOut * ncol, p.fft);
    else
      for (int l0 = 0; l0 < kOut * ncol; l0 += p.zgroup)
        lds_line_fft<1, T>(lds + l0 * ld, ld, min(p.zgroup, kOut * ncol - l0), p.fft);

    for (int l = wave; l < kOut * ncol; l += nwaves) {
      const int f = MULTI ? fdiv(l, p.fd_ncol) : l, c = MULTI ? l - f * ncol : 0;
      if (MULTI && c >= nct) continue;
      const rsrc_t rb = make_rsrc(p.b + (i64)f * p.npts, p.field_bytes);
      for (int z = p.z_lo + lane; z < p.z_hi; z += 64)
        gm<T>::stc(rb, (uint32_t)((col0 + c) * NZ + z), lds[l * ld + lpad(z)]);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ P3, two-stage lines
// The same pass for z-lines of N = RA * RB points with both radices known at
// compile time (one (kx, ky) column per tile).  Every LDS and global offset of a
// butterfly is then a constant from one base address, and the lines go
// straight from global memory into the registers of their first stage:
//   stage A (radix RA, RB butterflies per line): butterfly j of a line takes
//     x[j + RB t], t < RA, and its outputs go to the intermediate row j,
//     Y[j][t] (rows padded to PA = RA | 1 slots so that the lanes' rows fall in
//     different LDS banks);
//   stage B (radix RB, RA butterflies per line): butterfly j' takes column j'
//     of Y, Y[t'][j'] = y[j' + RA t'], applies w_N^(t' j'), and its outputs are
//     the transform at j' + RA t (natural order).
// The forward results of the 11 lines are written to LDS in natural order for
// the push; the 6 lines of E and B then run stage A from LDS and stage B
// straight to global memory (interior z only).  PML: the push writes the twelve
// split-part increments (a twelfth LDS line), and all twelve lines go back.
template <int RA, int RB>
struct TwoStage {
  static constexpr int N = RA * RB;
  static constexpr int PA = RA | 1;
  static constexpr int LD = two_stage_slots(RA, RB);  // LDS slots per line
};

template <typename T, int RA, int RB, int NTH, typename Src, bool PML = false>
__device__ __forceinline__ void zpush_two_stage_body(const Src& S) {
  using G = TwoStage<RA, RB>;
  constexpr int N = G::N, PA = G::PA, LD = G::LD;
  constexpr int kLines = PML ? 12 : 11, kOut = PML ? 12 : 6;  // LDS lines, lines transformed back
  cx<T>* lds = lds_base<T>();
  const int tid = threadIdx.x;
  // stage B twiddles w^(t k), copied once per launch to LDS as [t - 1][k] (lanes take consecutive k)
  Tw<T>* twl = reinterpret_cast<Tw<T>*>(lds + kLines * LD);
  {
    int col0;
    const ZPushParams<T>& p0 = S.box(blockIdx.x, col0);
    for (int i = tid; i < RA * (RB - 1); i += NTH) {
      const int k = i / (RB - 1), t = i - k * (RB - 1);
      twl[t * RA + k] = p0.fft.tw[(RA - 1) + i];
    }
    __syncthreads();
  }
  for (int tile = blockIdx.x; tile < S.ntiles(); tile += gridDim.x) {
    int col;
    const ZPushParams<T>& p = S.box(tile, col);
    // this thread's push coefficients (points tid and tid + NTH), loaded before the transforms
    constexpr int NP = (N + NTH - 1) / NTH;
    T cof[NP][5];
#pragma unroll
    for (int u = 0; u < NP; ++u)
#pragma unroll
      for (int k = 0; k < 5; ++k)
        cof[u][k] = gm<T>::ld(make_rsrc(p.coef + (i64)k * p.npts, p.coef_bytes),
                              u * NTH + tid < N ? (uint32_t)(col * N + u * NTH + tid) : kOOB);
    // forward stage A: global -> registers -> DFT -> intermediate rows
#pragma unroll
    for (int b0 = 0; b0 < 11 * RB; b0 += NTH) {
      const int b = b0 + tid;
      if (b0 + NTH <= 11 * RB || b < 11 * RB) {
        const int f = b / RB, j = b - f * RB;
        // plain global addresses: the lanes of a wave read several fields, which a
        // buffer resource (one base per wave) could only serve one field at a time
        const cx<T>* src = p.b + (i64)f * p.npts + (i64)col * N + j;
        cx<T> v[RA];
#pragma unroll
        for (int t = 0; t < RA; ++t) v[t] = src[RB * t];
        dft<RA, -1, T>::run(v);
        cx<T>* y = lds + f * LD + j * PA;
#pragma unroll
        for (int t = 0; t < RA; ++t) y[t] = v[t];
      }
    }
    __syncthreads();
    // forward stage B: intermediate columns -> twiddles -> DFT -> natural order (in place)
    {
      constexpr int NB = (11 * RA + NTH - 1) / NTH;
      cx<T> v[NB][RB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int b = u * NTH + tid;
        if (b < 11 * RA) {
          const int f = b / RA, k = b - f * RA;
          const cx<T>* y = lds + f * LD + k;
#pragma unroll
          for (int t = 0; t < RB; ++t) v[u][t] = y[t * PA];
          if (k > 0) {
#pragma unroll
            for (int t = 1; t < RB; ++t) v[u][t] = twmul<-1>(v[u][t], twl[(t - 1) * RA + k]);
          }
          dft<RB, -1, T>::run(v[u]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int b = u * NTH + tid;
        if (b < 11 * RA) {
          const int f = b / RA, k = b - f * RA;
          cx<T>* z = lds + f * LD + k;
#pragma unroll
          for (int t = 0; t < RB; ++t) z[t * RA] = v[u][t];
        }
      }
    }
    __syncthreads();
    // push, point by point (natural order, field f of point kz at f * LD + kz)
    {
      const int kxi = fdiv(col, p.fd_NY);
      const int kyi = col - kxi * p.NY;
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        const int kz = u * NTH + tid;
        if (kz < N) {
          if constexpr (PML)
            push_point_pml(p, lds, LD, kz, kz, kxi, kyi, cof[u]);
          else
            push_point_c(p, lds, LD, kz, kz, kxi, kyi, cof[u]);
        }
      }
    }
    __syncthreads();
    // inverse stage A on the 6 lines of E and B (PML: 12), from LDS (natural order) back to rows
    {
      constexpr int NA = (kOut * RB + NTH - 1) / NTH;
      cx<T> v[NA][RA];
#pragma unroll
      for (int u = 0; u < NA; ++u) {
        const int b = u * NTH + tid;
        if (b < kOut * RB) {
          const int f = b / RB, j = b - f * RB;
          const cx<T>* x = lds + f * LD + j;
#pragma unroll
          for (int t = 0; t < RA; ++t) v[u][t] = x[RB * t];
          dft<RA, 1, T>::run(v[u]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NA; ++u) {
        const int b = u * NTH + tid;
        if (b < kOut * RB) {
          const int f = b / RB, j = b - f * RB;
          cx<T>* y = lds + f * LD + j * PA;
#pragma unroll
          for (int t = 0; t < RA; ++t) y[t] = v[u][t];
        }
      }
    }
    __syncthreads();
    // inverse stage B: rows -> twiddles -> DFT -> global (interior z only)
#pragma unroll
    for (int b0 = 0; b0 < kOut * RA; b0 += NTH) {
      const int b = b0 + tid;
      if (b0 + NTH <= kOut * RA || b < kOut * RA) {
        const int f = b / RA, k = b - f * RA;
        const cx<T>* y = lds + f * LD + k;
        cx<T> v[RB];
#pragma unroll
        for (int t = 0; t < RB; ++t) v[t] = y[t * PA];
        if (k > 0) {
#pragma unroll
          for (int t = 1; t < RB; ++t) v[t] = twmul<1>(v[t], twl[(t - 1) * RA + k]);
        }
        dft<RB, 1, T>::run(v);
        cx<T>* dst = p.b + (i64)f * p.npts + (i64)col * N + k;
#pragma unroll
        for (int t = 0; t < RB; ++t) {
          const int z = k + RA * t;
          if (z >= p.z_lo && z < p.z_hi) dst[RA * t] = v[t];
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ P5
// Tiles are ty/2 complex x-lines rebuilt from the half spectra of ty real
// lines; loads go straight to LDS in rounds, several blocks per CU overlap.
template <typename T, typename Src>
__device__ __forceinline__ void xinv_body(const Src& S) {
  constexpr int kRound = load_round<T>::v / 2;  // two values per element
  cx<T>* lds = lds_base<T>();
  const int tid = threadIdx.x, nth = blockDim.x;

  for (int tile = blockIdx.x; tile < S.ntiles(); tile += gridDim.x) {
    int lt;
    const XInvParams<T>& p = S.box(tile, lt);
    const int q = fdiv(lt, p.fd_ytiles);
    const int ybase = p.y_lo + (lt - q * p.ytiles) * p.ty;
    const int f = fdiv(q, p.fd_nz);
    const int z = p.z_lo + (q - f * (p.z_hi - p.z_lo));
    const int NX = p.NX, NY = p.NY, NXH = p.NXH, nc = p.ty >> 1;
    const int ld = fft_slots(p.fft.sch.n);
    {
      // Rebuild Z = A + i B over the full line from the half spectra of the two real lines.
      const int nld = nc * NXH;
      const rsrc_t src = make_rsrc(p.src + (i64)f * p.npts, p.src_bytes);
      const int sbase = z * NXH * NY;
      Walk w;
      w.row = fdiv(tid, p.fd_nc);  // (kx, complex line)
      w.col = tid - w.row * nc;
      const int ldr = fdiv(nth, p.fd_nc), ldc = nth - ldr * nc;  // block stride over (kx, complex line)
      for (int e0 = 0; e0 < nld; e0 += kRound * nth) {
        cx<T> av[kRound], bv[kRound];
        Walk w0 = w;
#pragma unroll
        for (int u = 0; u < kRound; ++u) {
          uint32_t ia = kOOB, ib = kOOB;
          if (e0 + tid + u * nth < nld) {
            const int ya = ybase + 2 * w.col;
            if (ya < p.y_hi) ia = (uint32_t)(sbase + w.row * NY + ya);
            if (ya + 1 < p.y_hi) ib = (uint32_t)(sbase + w.row * NY + ya + 1);
          }
          av[u] = gm<T>::ldc(src, ia);
          bv[u] = gm<T>::ldc(src, ib);
          w.next(ldr, ldc, nc);
        }
#pragma unroll
        for (int u = 0; u < kRound; ++u) {
          if (e0 + tid + u * nth < nld) {
            const int kx = w0.row, c = w0.col;
            cx<T> x = av[u], y = bv[u];
            const bool selfconj = (kx == 0) || (2 * kx == NX);
            if (selfconj) {
              x.im = T(0);
              y.im = T(0);
            }
            lds[c * ld + lpad(kx)] = {x.re - y.im, x.im + y.re};
            if (!selfconj) lds[c * ld + lpad(NX - kx)] = {x.re + y.im, y.re - x.im};
          }
          w0.next(ldr, ldc, nc);
        }
      }
    }
    __syncthreads();
    lds_line_fft<1, T>(lds, ld, nc, p.fft);

    const rsrc_t dst = make_rsrc(p.dst[f], p.dst_bytes);
    const int zrow = p.scatter ? fmod_i(p.oz + z - p.gz, p.fd_GZ) * p.GY : z * NY;
    const int rowlen = p.scatter ? p.GX : NX;
    const int nwr = nc * NX;
    Walk v;
    v.row = fdiv(tid, p.fd_NX);  // (complex line, x)
    v.col = tid - v.row * NX;
    const int wdr = fdiv(nth, p.fd_NX), wdc = nth - wdr * NX;  // block stride over (complex line, x)
#pragma unroll 4
    for (int e = tid; e < nwr; e += nth) {
      const int c = v.row, n = v.col;
      const cx<T> val = lds[c * ld + lpad(n)];
      const int ya = ybase + 2 * c;
      uint32_t ia = kOOB, ib = kOOB;
      if (!p.scatter) {
        if (ya < p.y_hi) ia = (uint32_t)((zrow + ya) * rowlen + n);
        if (ya + 1 < p.y_hi) ib = (uint32_t)((zrow + ya + 1) * rowlen + n);
      } else if (n >= p.gx && n < p.gx + p.nx) {
        // the interior is no larger than the grid and its origin lies in it: one wrap at most
        const int xg = wrap_once(p.ox + n - p.gx, p.GX);
        const int ra = wrap_once(p.oy + ya - p.gy, p.GY);
        if (ya < p.y_hi) ia = (uint32_t)((zrow + ra) * rowlen + xg);
        if (ya + 1 < p.y_hi) ib = (uint32_t)((zrow + wrap_once(ra + 1, p.GY)) * rowlen + xg);
      }
      // streamed: G1 is read back by the next step's fill
      gm<T>::template st<kXStore<T>>(dst, ia, val.re);
      gm<T>::template st<kXStore<T>>(dst, ib, val.im);
      v.next(wdr, wdc, NX);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ kernels
// x forward: at most 128 registers in FP32 (two blocks per CU).
template <typename T>
__global__ void __launch_bounds__(kLineThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1)))
k_xfwd(XFwdParams<T>) {
  xfwd_body<T>(SingleSrc<XFwdParams<T>>{});
}
template <typename T>
__global__ void __launch_bounds__(kLineThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1)))
k_xfwd_b(BatchArgs<XFwdParams<T>> a) {
  xfwd_body<T>(BatchSrc<XFwdParams<T>>{a});
}
// y passes (single box): FP32 capped at 80 registers, three blocks per CU.  The
// spills this costs are cheaper than the lost latency hiding of two blocks.
template <int S, typename T>
__global__ void __launch_bounds__(kLineThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 1)))
k_ypass(YPassParams<T>) {
  ypass_body<S, T>(SingleSrc<YPassParams<T>>{});
}
template <int S, typename T>
__global__ void __launch_bounds__(kLineThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1)))
k_ypass_b(BatchArgs<YPassParams<T>> a) {
  ypass_body<S, T>(BatchSrc<YPassParams<T>>{a});
}
// z pass: FP32 single-box tiles fit 96 registers (5 waves per SIMD), batched ones 128 (4);
// FP64 256 (2).
template <typename T, int NTH, bool MULTI, bool PML = false>
__global__ void __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 2)))
k_zpush(ZPushParams<T>) {
  zpush_body<T, MULTI, SingleSrc<ZPushParams<T>>, PML>(SingleSrc<ZPushParams<T>>{});
}
// Two-stage z kernel: three 4-wave blocks per CU in FP32 (168 registers hold a
// stage's butterfly, its twiddles and the small-DFT temporaries without spills).
template <typename T, int RA, int RB, bool PML = false>
__global__ void __launch_bounds__(kZTwoStageThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1)))
k_zpush2(ZPushParams<T>) {
  zpush_two_stage_body<T, RA, RB, kZTwoStageThreads, SingleSrc<ZPushParams<T>>, PML>(SingleSrc<ZPushParams<T>>{});
}
template <typename T, int NTH>
__global__ void __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
k_zpush_b(BatchArgs<ZPushParams<T>> a) {
  zpush_body<T, true>(BatchSrc<ZPushParams<T>>{a});
}
// x inverse: at most 128 registers in FP32; 256-thread blocks (four per CU) unless
// the lines need the larger block.
template <typename T, int RA, int RB>
__global__ void __launch_bounds__(two_stage_x_threads(RA, RB))
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) k_xfwd2(XFwdParams<T>) {
  xfwd_two_stage_body<T, RA, RB, kXTwoStageLines, two_stage_x_threads(RA, RB)>(
      *(const XFwdParams<T>*)__builtin_amdgcn_kernarg_segment_ptr());
}
// x inverse, two-stage: 168 registers in FP32 (its stage A holds a butterfly across a
// barrier); the LDS of a tile already limits a CU to four blocks of three waves.
template <typename T, int RA, int RB>
__global__ void __launch_bounds__(two_stage_x_threads(RA, RB))
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1))) k_xinv2(XInvParams<T>) {
  xinv_two_stage_body<T, RA, RB, kXTwoStageLines, two_stage_x_threads(RA, RB)>(
      *(const XInvParams<T>*)__builtin_amdgcn_kernarg_segment_ptr());
}
template <int S, typename T, int RA, int RB>
__global__ void __launch_bounds__(two_stage_y_threads(RA, RB))
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) k_ypass2(YPassParams<T>) {
  ypass_two_stage_body<S, T, RA, RB, kYTwoStageLines, two_stage_y_threads(RA, RB)>(SingleSrc<YPassParams<T>>{});
}
template <typename T, int NTH>
__global__ void __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1)))
k_xinv(XInvParams<T>) {
  xinv_body<T>(SingleSrc<XInvParams<T>>{});
}
template <typename T, int NTH>
__global__ void __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1)))
k_xinv_b(BatchArgs<XInvParams<T>> a) {
  xinv_body<T>(BatchSrc<XInvParams<T>>{a});
}

template <typename T>
size_t cx_bytes() {
  return sizeof(cx<T>);
}

int num_cus() {
  static int n = 0;
  if (n == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      n = v;
    else
      n = 256;
  }
  return n;
}

// Persistent grid: as many blocks as can be resident at once (capped by the tile count).
// Opts in to more than 64 KB of dynamic LDS when needed (the plan checked the device limit).
template <typename K>
unsigned persistent_grid(K kernel, int threads, size_t lds, int ntiles) {
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess || per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 1;
  }
  const long long g = (long long)per_cu * num_cus();
  return (unsigned)(g < ntiles ? g : ntiles);
}

template <typename K, typename A>
void launch_persistent(K kernel, const A& arg, int threads, size_t lds, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return;
  const unsigned g = persistent_grid(kernel, threads, lds, ntiles);
  hipLaunchKernelGGL(kernel, dim3(g), dim3(threads), lds, s, arg);
}

}  // namespace

// ------------------------------------------------------------------ launchers
template <typename T>
size_t xfwd_lds(const XFwdParams<T>& p) {
  const size_t lines = (size_t)(p.ty / 2) * fft_slots(p.fft.sch.n) * cx_bytes<T>();
  return lines + (p.xtab ? (size_t)(p.NX + p.ty) * sizeof(int) : 0);
}
template <typename T>
size_t ypass_lds(const YPassParams<T>& p) {
  return (size_t)p.nl * fft_slots(p.fft.sch.n) * cx_bytes<T>();
}
template <typename T>
size_t zpush_lds(const ZPushParams<T>& p) {
  return (size_t)(p.pml ? 12 : 11) * p.ncol * fft_slots(p.fft.sch.n) * cx_bytes<T>();
}
template <typename T>
size_t xinv_lds(const XInvParams<T>& p) {
  return (size_t)(p.ty / 2) * fft_slots(p.fft.sch.n) * cx_bytes<T>();
}

template <typename T, int I = 0>
void launch_xfwd_two_stage_at(const XFwdParams<T>& p, hipStream_t s) {
  if constexpr (I < (int)(sizeof(kXTwoStage) / sizeof(kXTwoStage[0]))) {
    constexpr int RA = kXTwoStage[I][0], RB = kXTwoStage[I][1];
    if (p.ra == RA && p.rb == RB) {
      const size_t lds = (size_t)kXTwoStageLines * two_stage_slots(RA, RB) * cx_bytes<T>() +
                         (size_t)((RA * RB + 3) & ~3) * sizeof(int) + (size_t)RA * (RB - 1) * sizeof(Tw<T>);
      launch_persistent(k_xfwd2<T, RA, RB>, p, two_stage_x_threads(RA, RB), lds, p.ntiles, s);
      return;
    }
    launch_xfwd_two_stage_at<T, I + 1>(p, s);
  }
}
template <typename T, int I = 0>
void launch_xinv_two_stage_at(const XInvParams<T>& p, hipStream_t s) {
  if constexpr (I < (int)(sizeof(kXTwoStage) / sizeof(kXTwoStage[0]))) {
    constexpr int RA = kXTwoStage[I][0], RB = kXTwoStage[I][1];
    if (p.ra == RA && p.rb == RB) {
      const size_t lds =
          (size_t)kXTwoStageLines * two_stage_slots(RA, RB) * cx_bytes<T>() + (size_t)RA * (RB - 1) * sizeof(Tw<T>);
      launch_persistent(k_xinv2<T, RA, RB>, p, two_stage_x_threads(RA, RB), lds, p.ntiles, s);
      return;
    }
    launch_xinv_two_stage_at<T, I + 1>(p, s);
  }
}
template <typename T>
void launch_xfwd(const XFwdParams<T>& p, hipStream_t s) {
  if (p.ra > 0) {
    launch_xfwd_two_stage_at<T>(p, s);
    return;
  }
  launch_persistent(k_xfwd<T>, p, kLineThreads, xfwd_lds(p), p.ntiles, s);
}
template <typename T, int I = 0>
void launch_ypass_two_stage_at(const YPassParams<T>& p, int inverse, hipStream_t s) {
  if constexpr (I < (int)(sizeof(kYTwoStage) / sizeof(kYTwoStage[0]))) {
    constexpr int RA = kYTwoStage[I][0], RB = kYTwoStage[I][1];
    if (p.ra == RA && p.rb == RB) {
      const size_t lds = (size_t)kYTwoStageLines * two_stage_y_slots(RA, RB) * cx_bytes<T>() +
                         (size_t)RA * (RB - 1) * sizeof(Tw<T>);
      constexpr int nth = two_stage_y_threads(RA, RB);
      if (inverse)
        launch_persistent(k_ypass2<1, T, RA, RB>, p, nth, lds, p.ntiles, s);
      else
        launch_persistent(k_ypass2<-1, T, RA, RB>, p, nth, lds, p.ntiles, s);
      return;
    }
    launch_ypass_two_stage_at<T, I + 1>(p, inverse, s);
  }
}
template <typename T>
void launch_ypass(const YPassParams<T>& p, int inverse, hipStream_t s) {
  if (p.ra > 0) {
    launch_ypass_two_stage_at<T>(p, inverse, s);
    return;
  }
  if (inverse)
    launch_persistent(k_ypass<1, T>, p, kLineThreads, ypass_lds(p), p.ntiles, s);
  else
    launch_persistent(k_ypass<-1, T>, p, kLineThreads, ypass_lds(p), p.ntiles, s);
}
template <typename T, bool MULTI, bool PML>
void launch_zpush_cols(const ZPushParams<T>& p, int nthreads, hipStream_t s) {
  if (nthreads == kZThreads[0])
    launch_persistent(k_zpush<T, kZThreads[0], MULTI, PML>, p, nthreads, zpush_lds(p), p.ntiles, s);
  else
    launch_persistent(k_zpush<T, kZThreads[1], MULTI, PML>, p, nthreads, zpush_lds(p), p.ntiles, s);
}
// The run-time z kernels build as four units (single / multi-column, ordinary / PML), in
// parallel: each unit instantiates one pair, the others only declare it.
#if defined(PSATD_UNIT)
#if PSATD_UNIT != 3
extern template void launch_zpush_cols<float, false, false>(const ZPushParams<float>&, int, hipStream_t);
extern template void launch_zpush_cols<double, false, false>(const ZPushParams<double>&, int, hipStream_t);
#endif
#if PSATD_UNIT != 7
extern template void launch_zpush_cols<float, true, false>(const ZPushParams<float>&, int, hipStream_t);
extern template void launch_zpush_cols<double, true, false>(const ZPushParams<double>&, int, hipStream_t);
#endif
#if PSATD_UNIT != 8
extern template void launch_zpush_cols<float, false, true>(const ZPushParams<float>&, int, hipStream_t);
extern template void launch_zpush_cols<double, false, true>(const ZPushParams<double>&, int, hipStream_t);
#endif
#if PSATD_UNIT != 9
extern template void launch_zpush_cols<float, true, true>(const ZPushParams<float>&, int, hipStream_t);
extern template void launch_zpush_cols<double, true, true>(const ZPushParams<double>&, int, hipStream_t);
#endif
#endif
template <typename T, int I = 0>
void launch_two_stage_at(const ZPushParams<T>& p, hipStream_t s) {
  if constexpr (I < (int)(sizeof(kZTwoStage) / sizeof(kZTwoStage[0]))) {
    constexpr int RA = kZTwoStage[I][0], RB = kZTwoStage[I][1];
    if (p.ra == RA && p.rb == RB) {
      const size_t tw = (size_t)RA * (RB - 1) * sizeof(Tw<T>);
      const size_t line = (size_t)two_stage_slots(RA, RB) * cx_bytes<T>();
      if (p.pml)
        launch_persistent(k_zpush2<T, RA, RB, true>, p, kZTwoStageThreads, 12 * line + tw, p.ntiles, s);
      else
        launch_persistent(k_zpush2<T, RA, RB>, p, kZTwoStageThreads, 11 * line + tw, p.ntiles, s);
      return;
    }
    launch_two_stage_at<T, I + 1>(p, s);
  }
}
template <typename T>
void launch_zpush_two_stage(const ZPushParams<T>& p, hipStream_t s) {
  launch_two_stage_at<T>(p, s);
}
// Built as a unit of its own (the two-stage kernels compile in parallel with the rest).
#if defined(PSATD_UNIT) && PSATD_UNIT != 6
extern template void launch_zpush_two_stage<float>(const ZPushParams<float>&, hipStream_t);
extern template void launch_zpush_two_stage<double>(const ZPushParams<double>&, hipStream_t);
#endif
template <typename T>
void launch_zpush(const ZPushParams<T>& p, int nthreads, hipStream_t s) {
  if (p.pml && p.ra == 0) {  // split-field increments on the run-time kernels
    if (p.ncol == 1)
      launch_zpush_cols<T, false, true>(p, nthreads, s);
    else
      launch_zpush_cols<T, true, true>(p, nthreads, s);
    return;
  }
  if (p.ra > 0) {
    launch_zpush_two_stage<T>(p, s);
    return;
  }
  if (p.ncol == 1)
    launch_zpush_cols<T, false, false>(p, nthreads, s);
  else
    launch_zpush_cols<T, true, false>(p, nthreads, s);
}
template <typename T>
void launch_xinv(const XInvParams<T>& p, hipStream_t s) {
  if (p.ra > 0) {
    launch_xinv_two_stage_at<T>(p, s);
    return;
  }
  if (p.nthreads == kXInvThreads)
    launch_persistent(k_xinv<T, kXInvThreads>, p, kXInvThreads, xinv_lds(p), p.ntiles, s);
  else
    launch_persistent(k_xinv<T, kLineThreads>, p, kLineThreads, xinv_lds(p), p.ntiles, s);
}

template <typename T>
void launch_xfwd_batch(const BatchArgs<XFwdParams<T>>& a, size_t lds, hipStream_t s) {
  launch_persistent(k_xfwd_b<T>, a, kLineThreads, lds, a.total, s);
}
template <typename T>
void launch_ypass_batch(const BatchArgs<YPassParams<T>>& a, int inverse, size_t lds, hipStream_t s) {
  if (inverse)
    launch_persistent(k_ypass_b<1, T>, a, kLineThreads, lds, a.total, s);
  else
    launch_persistent(k_ypass_b<-1, T>, a, kLineThreads, lds, a.total, s);
}
template <typename T>
void launch_zpush_batch(const BatchArgs<ZPushParams<T>>& a, int nthreads, size_t lds, hipStream_t s) {
  if (nthreads == kZThreads[0])
    launch_persistent(k_zpush_b<T, kZThreads[0]>, a, nthreads, lds, a.total, s);
  else
    launch_persistent(k_zpush_b<T, kZThreads[1]>, a, nthreads, lds, a.total, s);
}
template <typename T>
void launch_xinv_batch(const BatchArgs<XInvParams<T>>& a, int nthreads, size_t lds, hipStream_t s) {
  if (nthreads == kXInvThreads)
    launch_persistent(k_xinv_b<T, kXInvThreads>, a, kXInvThreads, lds, a.total, s);
  else
    launch_persistent(k_xinv_b<T, kLineThreads>, a, kLineThreads, lds, a.total, s);
}


// Explicit instantiations.  The build compiles this file once per (pass, precision)
// unit (-DPSATD_UNIT=1..5 -DPSATD_REAL=float|double) so that the units compile in
// parallel; without PSATD_UNIT everything is instantiated here.
#define PSATD_INST_1(T)                                                                     \
  template void launch_xfwd<T>(const XFwdParams<T>&, hipStream_t);                          \
  template void launch_xfwd_batch<T>(const BatchArgs<XFwdParams<T>>&, size_t, hipStream_t); \
  template size_t xfwd_lds<T>(const XFwdParams<T>&);
#define PSATD_INST_2(T)                                                                               \
  template void launch_ypass<T>(const YPassParams<T>&, int, hipStream_t);                             \
  template void launch_ypass_batch<T>(const BatchArgs<YPassParams<T>>&, int, size_t, hipStream_t); \
  template size_t ypass_lds<T>(const YPassParams<T>&);
#define PSATD_INST_3(T)                                                   \
  template void launch_zpush<T>(const ZPushParams<T>&, int, hipStream_t); \
  template size_t zpush_lds<T>(const ZPushParams<T>&);                    \
  template void launch_zpush_cols<T, false, false>(const ZPushParams<T>&, int, hipStream_t);
#define PSATD_INST_7(T) template void launch_zpush_cols<T, true, false>(const ZPushParams<T>&, int, hipStream_t);
#define PSATD_INST_8(T) template void launch_zpush_cols<T, false, true>(const ZPushParams<T>&, int, hipStream_t);
#define PSATD_INST_9(T) template void launch_zpush_cols<T, true, true>(const ZPushParams<T>&, int, hipStream_t);
#define PSATD_INST_4(T) \
  template void launch_zpush_batch<T>(const BatchArgs<ZPushParams<T>>&, int, size_t, hipStream_t);
#define PSATD_INST_6(T) template void launch_zpush_two_stage<T>(const ZPushParams<T>&, hipStream_t);
#define PSATD_INST_5(T)                                                                     \
  template void launch_xinv<T>(const XInvParams<T>&, hipStream_t);                          \
  template void launch_xinv_batch<T>(const BatchArgs<XInvParams<T>>&, int, size_t, hipStream_t); \
  template size_t xinv_lds<T>(const XInvParams<T>&);
#define PSATD_CAT2(a, b) a##b
#define PSATD_CAT(a, b) PSATD_CAT2(a, b)
#if defined(PSATD_UNIT) && defined(PSATD_REAL)
PSATD_CAT(PSATD_INST_, PSATD_UNIT)(PSATD_REAL)
#else
#define PSATD_INST_ALL(T)                                                                          \
  PSATD_INST_1(T) PSATD_INST_2(T) PSATD_INST_3(T) PSATD_INST_4(T) PSATD_INST_5(T) PSATD_INST_6(T) \
  PSATD_INST_7(T) PSATD_INST_8(T) PSATD_INST_9(T)
PSATD_INST_ALL(float)
PSATD_INST_ALL(double)
#endif

}  // namespace psatd
