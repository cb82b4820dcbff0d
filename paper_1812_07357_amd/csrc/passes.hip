// The five passes of one PSATD step on a box (gfx950).
//
//   P1 k_xfwd   G1 (periodic gather, guard fill fused) or box reals -> x R2C -> layout A
//   P2 k_ypass  layout A -> y C2C forward -> layout B
//   P3 k_zpush  layout B -> z C2C forward, analytic push, z C2C inverse -> layout B (E, B)
//   P4 k_ypass  layout B -> y C2C inverse -> layout A (E, B)
//   P5 k_xinv   layout A -> x C2R -> box reals or G1 interior (guard merge fused)
//
// Sec. 1.1 of arXiv:1812.07357 (Fourier transform, analytic k-space update,
// inverse transform) and Sec. 2.5.2 (fill G2 guards from G1, copy the interior
// back).  The real-to-complex and complex-to-real x transforms pack two
// neighbouring real y-lines into one complex line: with z = a + i b,
//   A(k) = (Z(k) + conj Z(-k)) / 2,   B(k) = (Z(k) - conj Z(-k)) / (2 i),
// and the inverse rebuilds Z = A + i B over the full line from the half
// spectra (imaginary parts of the self-conjugate bins dropped).
//
// Every kernel is persistent and software-pipelined: a block loads tile t into
// registers, moves it to LDS, issues the loads of its next tile (they stay in
// flight while the LDS transform of tile t runs), writes tile t out, and
// repeats.  This keeps HBM busy during the LDS phase.  All global accesses go
// through buffer resources with hardware range checks (gmem.hpp); an index that
// is out of range by construction (kOOB) reads zero and drops writes.

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
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// ------------------------------------------------------------------ P1
template <typename T>
__global__ void __launch_bounds__(kLineThreads) k_xfwd(XFwdParams<T> p) {
  constexpr int PF = prefetch_budget<T>::v;
  cx<T>* lds = lds_base<T>();
  const int tid = threadIdx.x, nth = blockDim.x;
  const int NX = p.NX, NY = p.NY, NXH = p.NXH, ty = p.ty, nc = ty >> 1;
  const int ld = fft_slots(p.fft.sch.n);
  const int nld = nc * NX;    // complex inputs per tile
  const int nwr = NXH * ty;   // half-spectrum outputs per tile
  Walk w0, v0;
  w0.row = fdiv(tid, p.fd_NX);
  w0.col = tid - w0.row * NX;
  v0.row = fdiv(tid, p.fd_ty);
  v0.col = tid - v0.row * ty;
  T re[PF], im[PF];

  auto decode = [&](int tile, int& f, int& z, int& ybase) {
    const int q = fdiv(tile, p.fd_ytiles);
    ybase = (tile - q * p.ytiles) * ty;
    f = fdiv(q, p.fd_NZ);
    z = q - f * p.NZ;
  };
  auto issue = [&](int tile) {
    int f, z, ybase;
    decode(tile, f, z, ybase);
    const rsrc_t src = make_rsrc(p.src[f], p.src_bytes);
    const int zrow = p.gather ? fmod_i(p.z0 + z, p.fd_GZ) * p.GY : z * NY;
    const int rowlen = p.gather ? p.GX : NX;
    Walk w = w0;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int e = tid + u * nth;
      uint32_t ia = kOOB, ib = kOOB;
      if (e < nld) {
        const int ya = ybase + 2 * w.row;
        int xs = w.col, ra = ya, rb = ya + 1;
        if (p.gather) {
          xs = fmod_i(p.x0 + w.col, p.fd_GX);
          ra = fmod_i(p.y0 + ya, p.fd_GY);
          rb = fmod_i(p.y0 + ya + 1, p.fd_GY);
        }
        if (ya < NY) ia = (uint32_t)((zrow + ra) * rowlen + xs);
        if (ya + 1 < NY) ib = (uint32_t)((zrow + rb) * rowlen + xs);
      }
      re[u] = gm<T>::ld(src, ia);
      im[u] = gm<T>::ld(src, ib);
      w.next(p.ld_drow, p.ld_dcol, NX);
    }
  };

  int tile = blockIdx.x;
  if (tile >= p.ntiles) return;
  issue(tile);
  for (;;) {
    int f, z, ybase;
    decode(tile, f, z, ybase);
    {
      Walk w = w0;
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        if (tid + u * nth < nld) lds[w.row * ld + lpad(w.col)] = {re[u], im[u]};
        w.next(p.ld_drow, p.ld_dcol, NX);
      }
    }
    __syncthreads();
    const int next = tile + gridDim.x;
    if (next < p.ntiles) issue(next);
    lds_line_fft<-1, T>(lds, ld, nc, p.fft);

    // Split each complex line into the half spectra of its two real lines; y fastest.
    const rsrc_t dst = make_rsrc(p.dst + (i64)f * p.npts, p.dst_bytes);
    const int ny_t = min(ty, NY - ybase);
    Walk v = v0;
#pragma unroll 4
    for (int e = tid; e < nwr; e += nth) {
      const int kx = v.row, t = v.col;
      const int c = t >> 1;
      const cx<T> za = lds[c * ld + lpad(kx)];
      const cx<T> zb = cconj(lds[c * ld + lpad(kx == 0 ? 0 : NX - kx)]);
      cx<T> val;
      if ((t & 1) == 0) {
        val = cscale(cadd(za, zb), T(0.5));
      } else {
        const cx<T> d = csub(za, zb);
        val = {T(0.5) * d.im, T(-0.5) * d.re};
      }
      const uint32_t o = (t < ny_t) ? (uint32_t)((z * NXH + kx) * NY + ybase + t) : kOOB;
      gm<T>::stc(dst, o, val);
      v.next(p.wr_drow, p.wr_dcol, ty);
    }
    __syncthreads();
    if (next >= p.ntiles) break;
    tile = next;
  }
}

// ------------------------------------------------------------------ P2 / P4
template <int S, typename T>
__global__ void __launch_bounds__(kLineThreads) k_ypass(YPassParams<T> p) {
  constexpr int PF = prefetch_budget<T>::v;
  cx<T>* lds = lds_base<T>();
  const int tid = threadIdx.x, nth = blockDim.x;
  const int n = p.n;
  const int ld = fft_slots(p.fft.sch.n);
  // block strides of the two walk orders over a tile
  const int pn_drow = fdiv(nth, p.fd_n), pn_dcol = nth - pn_drow * n;  // positions fastest
  cx<T> r[PF];

  auto decode = [&](int tile, int& f, int& o, int& u0, int& nlt, FastDiv& fnl) {
    const int q = fdiv(tile, p.fd_utiles);
    const int ut = tile - q * p.utiles;
    f = fdiv(q, p.fd_nouter);
    o = q - f * p.nouter;
    u0 = p.u_lo + ut * p.nl;
    const bool last = (ut == p.utiles - 1);
    nlt = last ? p.nl_last : p.nl;
    fnl = last ? p.fd_nl_last : p.fd_nl;
  };
  // element e of a tile -> (line t, position q) in the input's preferred order
  auto start_in = [&](const FastDiv& fnl, int nlt, Walk& w, int& dr, int& dc) {
    if (p.ps_in == 1) {
      w.row = fdiv(tid, p.fd_n);
      w.col = tid - w.row * n;
      dr = pn_drow;
      dc = pn_dcol;
    } else {
      w.row = fdiv(tid, fnl);
      w.col = tid - w.row * nlt;
      dr = fdiv(nth, fnl);
      dc = nth - dr * nlt;
    }
  };
  auto issue = [&](int tile) {
    int f, o, u0, nlt;
    FastDiv fnl;
    decode(tile, f, o, u0, nlt, fnl);
    const rsrc_t in = make_rsrc(p.in + (i64)f * p.fs_in, p.in_bytes);
    const int base = o * p.os_in + u0 * p.ls_in;
    const int tot = nlt * n;
    Walk w;
    int dr, dc;
    start_in(fnl, nlt, w, dr, dc);
    const int ncol = (p.ps_in == 1) ? n : nlt;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      uint32_t idx = kOOB;
      if (tid + u * nth < tot) {
        const int t = (p.ps_in == 1) ? w.row : w.col;
        const int q = (p.ps_in == 1) ? w.col : w.row;
        idx = (uint32_t)(base + t * p.ls_in + q * p.ps_in);
      }
      r[u] = gm<T>::ldc(in, idx);
      w.next(dr, dc, ncol);
    }
  };

  int tile = blockIdx.x;
  if (tile >= p.ntiles) return;
  issue(tile);
  for (;;) {
    int f, o, u0, nlt;
    FastDiv fnl;
    decode(tile, f, o, u0, nlt, fnl);
    {
      Walk w;
      int dr, dc;
      start_in(fnl, nlt, w, dr, dc);
      const int ncol = (p.ps_in == 1) ? n : nlt;
      const int tot = nlt * n;
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        if (tid + u * nth < tot) {
          const int t = (p.ps_in == 1) ? w.row : w.col;
          const int q = (p.ps_in == 1) ? w.col : w.row;
          lds[t * ld + lpad(q)] = r[u];
        }
        w.next(dr, dc, ncol);
      }
    }
    __syncthreads();
    const int next = tile + gridDim.x;
    if (next < p.ntiles) issue(next);
    lds_line_fft<S, T>(lds, ld, nlt, p.fft);

    const rsrc_t out = make_rsrc(p.out + (i64)f * p.fs_out, p.out_bytes);
    const int obase = o * p.os_out + u0 * p.ls_out;
    const int np = p.p_hi - p.p_lo;
    const int tot = nlt * np;
    Walk w;
    int dr, dc, ncol;
    if (p.ps_out == 1) {
      w.row = fdiv(tid, p.fd_np);
      w.col = tid - w.row * np;
      dr = fdiv(nth, p.fd_np);
      dc = nth - dr * np;
      ncol = np;
    } else {
      w.row = fdiv(tid, fnl);
      w.col = tid - w.row * nlt;
      dr = fdiv(nth, fnl);
      dc = nth - dr * nlt;
      ncol = nlt;
    }
#pragma unroll 4
    for (int e = tid; e < tot; e += nth) {
      const int t = (p.ps_out == 1) ? w.row : w.col;
      const int q = p.p_lo + ((p.ps_out == 1) ? w.col : w.row);
      gm<T>::stc(out, (uint32_t)(obase + t * p.ls_out + q * p.ps_out), lds[t * ld + lpad(q)]);
      w.next(dr, dc, ncol);
    }
    __syncthreads();
    if (next >= p.ntiles) break;
    tile = next;
  }
}

// ------------------------------------------------------------------ P3
// Push (Sec. 1.1; J constant over the step, rho at both ends):
//   E' = C E + i c^2 S1 (K x B) - (S1/eps0) J + i (c^2/eps0) K (X3 rho_old - X2 rho_new)
//   B' = C B - i S1 (K x E) + i (X1/eps0) (K x J)
// Each wave moves whole z-lines (lines w, w + nwaves, ...), so the field of a
// wave's load is uniform and one buffer resource serves it.
constexpr int kZPts = 2;  // k-space points per thread in the push (NZ <= kZPts * threads)

template <typename T, int NTH>
__global__ void __launch_bounds__(NTH) k_zpush(ZPushParams<T> p) {
  constexpr int PF = prefetch_budget<T>::v;
  cx<T>* lds = lds_base<T>();
  const int tid = threadIdx.x, nth = blockDim.x;
  const int lane = tid & 63;
  const int wave = uniform(tid >> 6);
  const int nwaves = nth >> 6;
  const int NZ = p.NZ;
  const int ld = fft_slots(p.fft.sch.n);
  const int per_line = (NZ + 63) >> 6;
  cx<T> r[PF];
  T cc[kZPts][5], kzv[kZPts];
#pragma unroll
  for (int q = 0; q < kZPts; ++q) {
    const int kz = tid + q * nth;
    kzv[q] = kz < NZ ? p.kz[kz] : T(0);
  }
  rsrc_t ct[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) ct[i] = make_rsrc(p.coef + (i64)i * p.npts, p.coef_bytes);

  // slot u of the prefetch = (this wave's line number s, chunk i): line wave + s*nwaves, z = lane + 64 i
  auto issue_fields = [&](int col) {
    int s = 0, i = 0;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int l = wave + s * nwaves;
      const rsrc_t rb = make_rsrc(p.b + (i64)(l < 11 ? l : 0) * p.npts, p.field_bytes);
      const int z = lane + 64 * i;
      const uint32_t idx = (l < 11 && z < NZ) ? (uint32_t)(col * NZ + z) : kOOB;
      r[u] = gm<T>::ldc(rb, idx);
      if (++i == per_line) {
        i = 0;
        ++s;
      }
    }
  };
  auto drain_fields = [&]() {
    int s = 0, i = 0;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int l = wave + s * nwaves;
      const int z = lane + 64 * i;
      if (l < 11 && z < NZ) lds[l * ld + lpad(z)] = r[u];
      if (++i == per_line) {
        i = 0;
        ++s;
      }
    }
  };
  auto issue_coefs = [&](int col) {
#pragma unroll
    for (int q = 0; q < kZPts; ++q) {
      const int kz = tid + q * nth;
      const uint32_t idx = kz < NZ ? (uint32_t)(col * NZ + kz) : kOOB;
#pragma unroll
      for (int i = 0; i < 5; ++i) cc[q][i] = gm<T>::ld(ct[i], idx);
    }
  };

  int col = blockIdx.x;
  if (col >= p.ncols) return;
  issue_fields(col);
  issue_coefs(col);
  for (;;) {
    drain_fields();
    __syncthreads();
    const int next = col + gridDim.x;
    lds_line_fft<-1, T>(lds, ld, 11, p.fft);

    const int kxi = fdiv(col, p.fd_NY);
    const int kyi = col - kxi * p.NY;
    const T kx = p.kx[kxi];
    const T ky = p.ky[kyi];
    const T c2 = p.c2, ie = p.inv_eps0;
#pragma unroll
    for (int q = 0; q < kZPts; ++q) {
      const int kz = tid + q * nth;
      if (kz >= NZ) continue;
      const T C = cc[q][0], S1 = cc[q][1], X1 = cc[q][2], X2 = cc[q][3], X3 = cc[q][4];
      const T kzz = kzv[q];
      const int s = lpad(kz);
      const cx<T> ex = lds[0 * ld + s], ey = lds[1 * ld + s], ez = lds[2 * ld + s];
      const cx<T> bx = lds[3 * ld + s], by = lds[4 * ld + s], bz = lds[5 * ld + s];
      const cx<T> jx = lds[6 * ld + s], jy = lds[7 * ld + s], jz = lds[8 * ld + s];
      const cx<T> ro = lds[9 * ld + s], rn = lds[10 * ld + s];
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
      lds[0 * ld + s] = {C * ex.re - sj * jx.re - ux.im, C * ex.im - sj * jx.im + ux.re};
      lds[1 * ld + s] = {C * ey.re - sj * jy.re - uy.im, C * ey.im - sj * jy.im + uy.re};
      lds[2 * ld + s] = {C * ez.re - sj * jz.re - uz.im, C * ez.im - sj * jz.im + uz.re};
      // B' = C B + i (xj K x J - S1 K x E)
      const cx<T> wx = csub(cscale(kjx, xj), cscale(kex, S1));
      const cx<T> wy = csub(cscale(kjy, xj), cscale(key, S1));
      const cx<T> wz = csub(cscale(kjz, xj), cscale(kez, S1));
      lds[3 * ld + s] = {C * bx.re - wx.im, C * bx.im + wx.re};
      lds[4 * ld + s] = {C * by.re - wy.im, C * by.im + wy.re};
      lds[5 * ld + s] = {C * bz.re - wz.im, C * bz.im + wz.re};
    }
    // The next column's loads fly during the inverse transform and the stores
    // (issued here rather than before the push to keep the push's registers free).
    if (next < p.ncols) {
      issue_coefs(next);
      issue_fields(next);
    }
    __syncthreads();
    lds_line_fft<1, T>(lds, ld, 6, p.fft);

    for (int l = wave; l < 6; l += nwaves) {
      const rsrc_t rb = make_rsrc(p.b + (i64)l * p.npts, p.field_bytes);
      for (int z = p.z_lo + lane; z < p.z_hi; z += 64) gm<T>::stc(rb, (uint32_t)(col * NZ + z), lds[l * ld + lpad(z)]);
    }
    __syncthreads();
    if (next >= p.ncols) break;
    col = next;
  }
}

// ------------------------------------------------------------------ P5
template <typename T>
__global__ void __launch_bounds__(kLineThreads) k_xinv(XInvParams<T> p) {
  constexpr int PF2 = prefetch_budget<T>::v / 2;  // two values per element
  cx<T>* lds = lds_base<T>();
  const int tid = threadIdx.x, nth = blockDim.x;
  const int NX = p.NX, NXH = p.NXH, NY = p.NY, ty = p.ty, nc = ty >> 1;
  const int ld = fft_slots(p.fft.sch.n);
  const int nld = nc * NXH;
  const int nwr = nc * NX;
  Walk w0, v0;
  w0.row = fdiv(tid, p.fd_nc);  // (kx, complex line)
  w0.col = tid - w0.row * nc;
  v0.row = fdiv(tid, p.fd_NX);  // (complex line, x)
  v0.col = tid - v0.row * NX;
  cx<T> a[PF2], b[PF2];

  auto decode = [&](int tile, int& f, int& z, int& ybase) {
    const int q = fdiv(tile, p.fd_ytiles);
    ybase = p.y_lo + (tile - q * p.ytiles) * ty;
    f = fdiv(q, p.fd_nz);
    z = p.z_lo + (q - f * (p.z_hi - p.z_lo));
  };
  auto issue = [&](int tile) {
    int f, z, ybase;
    decode(tile, f, z, ybase);
    const rsrc_t src = make_rsrc(p.src + (i64)f * p.npts, p.src_bytes);
    const int sbase = z * NXH * NY;
    Walk w = w0;
#pragma unroll
    for (int u = 0; u < PF2; ++u) {
      uint32_t ia = kOOB, ib = kOOB;
      if (tid + u * nth < nld) {
        const int ya = ybase + 2 * w.col;
        if (ya < p.y_hi) ia = (uint32_t)(sbase + w.row * NY + ya);
        if (ya + 1 < p.y_hi) ib = (uint32_t)(sbase + w.row * NY + ya + 1);
      }
      a[u] = gm<T>::ldc(src, ia);
      b[u] = gm<T>::ldc(src, ib);
      w.next(p.ld_drow, p.ld_dcol, nc);
    }
  };

  int tile = blockIdx.x;
  if (tile >= p.ntiles) return;
  issue(tile);
  for (;;) {
    int f, z, ybase;
    decode(tile, f, z, ybase);
    {
      // Rebuild Z = A + i B over the full line from the half spectra of the two real lines.
      Walk w = w0;
#pragma unroll
      for (int u = 0; u < PF2; ++u) {
        if (tid + u * nth < nld) {
          const int kx = w.row, c = w.col;
          cx<T> av = a[u], bv = b[u];
          const bool selfconj = (kx == 0) || (2 * kx == NX);
          if (selfconj) {
            av.im = T(0);
            bv.im = T(0);
          }
          lds[c * ld + lpad(kx)] = {av.re - bv.im, av.im + bv.re};
          if (!selfconj) lds[c * ld + lpad(NX - kx)] = {av.re + bv.im, bv.re - av.im};
        }
        w.next(p.ld_drow, p.ld_dcol, nc);
      }
    }
    __syncthreads();
    const int next = tile + gridDim.x;
    if (next < p.ntiles) issue(next);
    lds_line_fft<1, T>(lds, ld, nc, p.fft);

    const rsrc_t dst = make_rsrc(p.dst[f], p.dst_bytes);
    const int zrow = p.scatter ? fmod_i(p.oz + z - p.gz, p.fd_GZ) * p.GY : z * NY;
    const int rowlen = p.scatter ? p.GX : NX;
    Walk v = v0;
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
        const int xg = fmod_i(p.ox + n - p.gx, p.fd_GX);
        if (ya < p.y_hi) ia = (uint32_t)((zrow + fmod_i(p.oy + ya - p.gy, p.fd_GY)) * rowlen + xg);
        if (ya + 1 < p.y_hi) ib = (uint32_t)((zrow + fmod_i(p.oy + ya + 1 - p.gy, p.fd_GY)) * rowlen + xg);
      }
      gm<T>::st(dst, ia, val.re);
      gm<T>::st(dst, ib, val.im);
      v.next(p.wr_drow, p.wr_dcol, NX);
    }
    __syncthreads();
    if (next >= p.ntiles) break;
    tile = next;
  }
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
  if (lds > 64 * 1024) (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess || per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 1;
  }
  const long long g = (long long)per_cu * num_cus();
  return (unsigned)(g < ntiles ? g : ntiles);
}

}  // namespace

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_xfwd(const XFwdParams<T>& p, hipStream_t s) {
  const size_t lds = (size_t)(p.ty / 2) * fft_slots(p.fft.sch.n) * cx_bytes<T>();
  const unsigned g = persistent_grid(k_xfwd<T>, kLineThreads, lds, p.ntiles);
  hipLaunchKernelGGL(k_xfwd<T>, dim3(g), dim3(kLineThreads), lds, s, p);
}

template <typename T>
void launch_ypass(const YPassParams<T>& p, int inverse, hipStream_t s) {
  const size_t lds = (size_t)p.nl * fft_slots(p.fft.sch.n) * cx_bytes<T>();
  if (inverse) {
    const unsigned g = persistent_grid(k_ypass<1, T>, kLineThreads, lds, p.ntiles);
    hipLaunchKernelGGL((k_ypass<1, T>), dim3(g), dim3(kLineThreads), lds, s, p);
  } else {
    const unsigned g = persistent_grid(k_ypass<-1, T>, kLineThreads, lds, p.ntiles);
    hipLaunchKernelGGL((k_ypass<-1, T>), dim3(g), dim3(kLineThreads), lds, s, p);
  }
}

template <typename T>
void launch_zpush(const ZPushParams<T>& p, int nthreads, hipStream_t s) {
  const size_t lds = (size_t)11 * fft_slots(p.fft.sch.n) * cx_bytes<T>();
  if (nthreads == kLineThreads) {
    const unsigned g = persistent_grid(k_zpush<T, kLineThreads>, nthreads, lds, p.ncols);
    hipLaunchKernelGGL((k_zpush<T, kLineThreads>), dim3(g), dim3(nthreads), lds, s, p);
  } else {
    const unsigned g = persistent_grid(k_zpush<T, 2 * kLineThreads>, nthreads, lds, p.ncols);
    hipLaunchKernelGGL((k_zpush<T, 2 * kLineThreads>), dim3(g), dim3(nthreads), lds, s, p);
  }
}

template <typename T>
void launch_xinv(const XInvParams<T>& p, hipStream_t s) {
  const size_t lds = (size_t)(p.ty / 2) * fft_slots(p.fft.sch.n) * cx_bytes<T>();
  const unsigned g = persistent_grid(k_xinv<T>, kLineThreads, lds, p.ntiles);
  hipLaunchKernelGGL(k_xinv<T>, dim3(g), dim3(kLineThreads), lds, s, p);
}

int zpush_points_per_thread() { return kZPts; }

template void launch_xfwd<float>(const XFwdParams<float>&, hipStream_t);
template void launch_xfwd<double>(const XFwdParams<double>&, hipStream_t);
template void launch_ypass<float>(const YPassParams<float>&, int, hipStream_t);
template void launch_ypass<double>(const YPassParams<double>&, int, hipStream_t);
template void launch_zpush<float>(const ZPushParams<float>&, int, hipStream_t);
template void launch_zpush<double>(const ZPushParams<double>&, int, hipStream_t);
template void launch_xinv<float>(const XInvParams<float>&, hipStream_t);
template void launch_xinv<double>(const XInvParams<double>&, hipStream_t);

}  // namespace psatd
