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
// Every global access is bounds-checked against the buffer extent; an
// out-of-range index reads zero / skips the write instead of faulting.

#include "internal.hpp"

namespace psatd {

namespace {

constexpr int kThreads = 256;

__host__ __device__ inline int lds_stride(int n) { return n + ((n & 1) ? 0 : 1); }

template <typename T>
__device__ inline cx<T>* lds_base() {
  extern __shared__ double2 psatd_smem[];
  return reinterpret_cast<cx<T>*>(psatd_smem);
}

template <typename T>
__device__ inline T ld_chk(const T* p, i64 i, i64 n) {
  return (i >= 0 && i < n) ? p[i] : T(0);
}
template <typename T>
__device__ inline cx<T> ld_chk(const cx<T>* p, i64 i, i64 n) {
  return (i >= 0 && i < n) ? p[i] : cx<T>{T(0), T(0)};
}
template <typename T>
__device__ inline void st_chk(T* p, i64 i, i64 n, T v) {
  if (i >= 0 && i < n) p[i] = v;
}

// ------------------------------------------------------------------ P1
template <typename T>
__global__ void __launch_bounds__(kThreads) k_xfwd(XFwdParams<T> p) {
  cx<T>* lds = lds_base<T>();
  const int f = blockIdx.y;
  const int tile = blockIdx.x % p.ytiles;
  const int z = blockIdx.x / p.ytiles;
  const int ybase = tile * p.ty;
  const int nc = p.ty >> 1;
  const int NX = p.NX;
  const int ld = lds_stride(NX);
  const T* __restrict__ src = p.src[f];
  const int nth = blockDim.x;

  // Row offsets of the two real lines of complex line c are recomputed per element;
  // the gather wraps every index into the periodic global grid.
  for (int e = threadIdx.x; e < nc * NX; e += nth) {
    const int c = e / NX;
    const int n = e - c * NX;
    const int ya = ybase + 2 * c;
    const int yb = ya + 1;
    T re = T(0), im = T(0);
    if (p.gather) {
      const i64 zg = (p.z0 + z) % p.GZ;
      const i64 xg = (p.x0 + n) % p.GX;
      if (ya < p.NY) re = ld_chk(src, (zg * p.GY + (p.y0 + ya) % p.GY) * p.GX + xg, p.src_extent);
      if (yb < p.NY) im = ld_chk(src, (zg * p.GY + (p.y0 + yb) % p.GY) * p.GX + xg, p.src_extent);
    } else {
      if (ya < p.NY) re = ld_chk(src, ((i64)z * p.NY + ya) * NX + n, p.src_extent);
      if (yb < p.NY) im = ld_chk(src, ((i64)z * p.NY + yb) * NX + n, p.src_extent);
    }
    lds[c * ld + n] = {re, im};
  }
  __syncthreads();
  lds_fft<-1, T>(lds, ld, nc, p.sch, p.tw);

  cx<T>* __restrict__ dst = p.dst + (i64)f * p.NZ * p.NXH * p.NY;
  const i64 dext = p.dst_extent - (i64)f * p.NZ * p.NXH * p.NY;
  for (int e = threadIdx.x; e < p.NXH * p.ty; e += nth) {
    const int t = e % p.ty;
    const int kx = e / p.ty;
    const int y = ybase + t;
    if (y >= p.NY) continue;
    const int c = t >> 1;
    const cx<T> Z = lds[c * ld + kx];
    const cx<T> Zm = cconj(lds[c * ld + (kx == 0 ? 0 : NX - kx)]);
    cx<T> v;
    if ((t & 1) == 0) {
      v = cscale(cadd(Z, Zm), T(0.5));
    } else {
      const cx<T> d = csub(Z, Zm);
      v = {T(0.5) * d.im, T(-0.5) * d.re};
    }
    const i64 o = ((i64)z * p.NXH + kx) * p.NY + y;
    if (o < dext) dst[o] = v;
  }
}

// ------------------------------------------------------------------ P2 / P4
template <int S, typename T>
__global__ void __launch_bounds__(kThreads) k_ypass(YPassParams<T> p) {
  cx<T>* lds = lds_base<T>();
  const int f = blockIdx.y;
  const int ut = blockIdx.x % p.utiles;
  const int o = blockIdx.x / p.utiles;
  const int u0 = p.u_lo + ut * p.nl;
  const int nl = min(p.nl, p.u_hi - u0);
  const int n = p.n;
  const int ld = lds_stride(n);
  const int nth = blockDim.x;
  const i64 ibase = (i64)f * p.fs_in + (i64)o * p.os_in + (i64)u0 * p.ls_in;
  const i64 obase = (i64)f * p.fs_out + (i64)o * p.os_out + (i64)u0 * p.ls_out;

  if (p.ps_in == 1) {
    for (int e = threadIdx.x; e < nl * n; e += nth) {
      const int t = e / n;
      const int q = e - t * n;
      lds[t * ld + q] = ld_chk(p.in, ibase + (i64)t * p.ls_in + q, p.in_extent);
    }
  } else {
    for (int e = threadIdx.x; e < nl * n; e += nth) {
      const int t = e % nl;
      const int q = e / nl;
      lds[t * ld + q] = ld_chk(p.in, ibase + (i64)t * p.ls_in + (i64)q * p.ps_in, p.in_extent);
    }
  }
  __syncthreads();
  lds_fft<S, T>(lds, ld, nl, p.sch, p.tw);

  const int np = p.p_hi - p.p_lo;
  if (p.ps_out == 1) {
    for (int e = threadIdx.x; e < nl * np; e += nth) {
      const int t = e / np;
      const int q = p.p_lo + (e - t * np);
      const i64 oi = obase + (i64)t * p.ls_out + q;
      if (oi < p.out_extent) p.out[oi] = lds[t * ld + q];
    }
  } else {
    for (int e = threadIdx.x; e < nl * np; e += nth) {
      const int t = e % nl;
      const int q = p.p_lo + e / nl;
      const i64 oi = obase + (i64)t * p.ls_out + (i64)q * p.ps_out;
      if (oi < p.out_extent) p.out[oi] = lds[t * ld + q];
    }
  }
}

// ------------------------------------------------------------------ P3
// Push (Sec. 1.1; J constant over the step, rho at both ends):
//   E' = C E + i c^2 S1 (K x B) - (S1/eps0) J + i (c^2/eps0) K (X3 rho_old - X2 rho_new)
//   B' = C B - i S1 (K x E) + i (X1/eps0) (K x J)
template <typename T>
__global__ void __launch_bounds__(2 * kThreads) k_zpush(ZPushParams<T> p) {
  cx<T>* lds = lds_base<T>();
  const i64 col = blockIdx.x;
  const int kxi = (int)(col / p.NY);
  const int kyi = (int)(col - (i64)kxi * p.NY);
  const int NZ = p.NZ;
  const int ld = lds_stride(NZ);
  const int nth = blockDim.x;
  const i64 ext = 11 * p.npts;

  for (int e = threadIdx.x; e < 11 * NZ; e += nth) {
    const int fz = e / NZ;
    const int z = e - fz * NZ;
    lds[fz * ld + z] = ld_chk(p.b, (i64)fz * p.npts + col * NZ + z, ext);
  }
  __syncthreads();
  lds_fft<-1, T>(lds, ld, 11, p.sch, p.tw);

  const T kx = p.kx[kxi];
  const T ky = p.ky[kyi];
  const T c2 = p.c2, ie = p.inv_eps0;
  for (int kz = threadIdx.x; kz < NZ; kz += nth) {
    const i64 q = col * NZ + kz;
    const T C = ld_chk(p.coef, q, 5 * p.npts);
    const T S1 = ld_chk(p.coef, p.npts + q, 5 * p.npts);
    const T X1 = ld_chk(p.coef, 2 * p.npts + q, 5 * p.npts);
    const T X2 = ld_chk(p.coef, 3 * p.npts + q, 5 * p.npts);
    const T X3 = ld_chk(p.coef, 4 * p.npts + q, 5 * p.npts);
    const T kzv = p.kz[kz];
    const cx<T> ex = lds[0 * ld + kz], ey = lds[1 * ld + kz], ez = lds[2 * ld + kz];
    const cx<T> bx = lds[3 * ld + kz], by = lds[4 * ld + kz], bz = lds[5 * ld + kz];
    const cx<T> jx = lds[6 * ld + kz], jy = lds[7 * ld + kz], jz = lds[8 * ld + kz];
    const cx<T> ro = lds[9 * ld + kz], rn = lds[10 * ld + kz];
    // K x B, K x E, K x J (K real)
    const cx<T> kbx = csub(cscale(bz, ky), cscale(by, kzv));
    const cx<T> kby = csub(cscale(bx, kzv), cscale(bz, kx));
    const cx<T> kbz = csub(cscale(by, kx), cscale(bx, ky));
    const cx<T> kex = csub(cscale(ez, ky), cscale(ey, kzv));
    const cx<T> key = csub(cscale(ex, kzv), cscale(ez, kx));
    const cx<T> kez = csub(cscale(ey, kx), cscale(ex, ky));
    const cx<T> kjx = csub(cscale(jz, ky), cscale(jy, kzv));
    const cx<T> kjy = csub(cscale(jx, kzv), cscale(jz, kx));
    const cx<T> kjz = csub(cscale(jy, kx), cscale(jx, ky));
    const cx<T> r = csub(cscale(ro, X3), cscale(rn, X2));
    const T a = c2 * S1;      // multiplies K x B
    const T g = c2 * ie;      // multiplies K r
    const T sj = S1 * ie;     // multiplies J
    const T xj = X1 * ie;     // multiplies K x J
    // E' = C E - sj J + i (a K x B + g K r)
    const cx<T> ux = cadd(cscale(kbx, a), cscale(r, g * kx));
    const cx<T> uy = cadd(cscale(kby, a), cscale(r, g * ky));
    const cx<T> uz = cadd(cscale(kbz, a), cscale(r, g * kzv));
    lds[0 * ld + kz] = {C * ex.re - sj * jx.re - ux.im, C * ex.im - sj * jx.im + ux.re};
    lds[1 * ld + kz] = {C * ey.re - sj * jy.re - uy.im, C * ey.im - sj * jy.im + uy.re};
    lds[2 * ld + kz] = {C * ez.re - sj * jz.re - uz.im, C * ez.im - sj * jz.im + uz.re};
    // B' = C B + i (xj K x J - S1 K x E)
    const cx<T> wx = csub(cscale(kjx, xj), cscale(kex, S1));
    const cx<T> wy = csub(cscale(kjy, xj), cscale(key, S1));
    const cx<T> wz = csub(cscale(kjz, xj), cscale(kez, S1));
    lds[3 * ld + kz] = {C * bx.re - wx.im, C * bx.im + wx.re};
    lds[4 * ld + kz] = {C * by.re - wy.im, C * by.im + wy.re};
    lds[5 * ld + kz] = {C * bz.re - wz.im, C * bz.im + wz.re};
  }
  __syncthreads();
  lds_fft<1, T>(lds, ld, 6, p.sch, p.tw);

  const int nz_out = p.z_hi - p.z_lo;
  for (int e = threadIdx.x; e < 6 * nz_out; e += nth) {
    const int fz = e / nz_out;
    const int z = p.z_lo + (e - fz * nz_out);
    const i64 oi = (i64)fz * p.npts + col * NZ + z;
    if (oi < ext) p.b[oi] = lds[fz * ld + z];
  }
}

// ------------------------------------------------------------------ P5
template <typename T>
__global__ void __launch_bounds__(kThreads) k_xinv(XInvParams<T> p) {
  cx<T>* lds = lds_base<T>();
  const int f = blockIdx.y;
  const int tile = blockIdx.x % p.ytiles;
  const int z = p.z_lo + blockIdx.x / p.ytiles;
  const int ybase = p.y_lo + tile * p.ty;
  const int nc = p.ty >> 1;
  const int NX = p.NX, NXH = p.NXH, NY = p.NY;
  const int ld = lds_stride(NX);
  const int nth = blockDim.x;
  const i64 sbase = ((i64)f * p.NZ + z) * NXH * NY;

  for (int e = threadIdx.x; e < nc * NXH; e += nth) {
    const int c = e % nc;
    const int kx = e / nc;
    const int ya = ybase + 2 * c;
    const int yb = ya + 1;
    cx<T> a = {T(0), T(0)}, b = {T(0), T(0)};
    if (ya < p.y_hi) a = ld_chk(p.src, sbase + (i64)kx * NY + ya, p.src_extent);
    if (yb < p.y_hi) b = ld_chk(p.src, sbase + (i64)kx * NY + yb, p.src_extent);
    const bool selfconj = (kx == 0) || (2 * kx == NX);
    if (selfconj) {
      a.im = T(0);
      b.im = T(0);
    }
    lds[c * ld + kx] = {a.re - b.im, a.im + b.re};
    if (!selfconj) lds[c * ld + (NX - kx)] = {a.re + b.im, b.re - a.im};
  }
  __syncthreads();
  lds_fft<1, T>(lds, ld, nc, p.sch, p.tw);

  T* __restrict__ dst = p.dst[f];
  for (int e = threadIdx.x; e < nc * NX; e += nth) {
    const int c = e / NX;
    const int n = e - c * NX;
    const cx<T> v = lds[c * ld + n];
    const int ya = ybase + 2 * c;
    if (!p.scatter) {
      if (ya < p.y_hi) st_chk(dst, ((i64)z * NY + ya) * NX + n, p.dst_extent, v.re);
      if (ya + 1 < p.y_hi) st_chk(dst, ((i64)z * NY + ya + 1) * NX + n, p.dst_extent, v.im);
    } else if (n >= p.gx && n < p.gx + p.nx) {
      const i64 zg = (p.oz + z - p.gz) % p.GZ;
      const i64 xg = (p.ox + n - p.gx) % p.GX;
      if (ya < p.y_hi)
        st_chk(dst, (zg * p.GY + (p.oy + ya - p.gy) % p.GY) * p.GX + xg, p.dst_extent, v.re);
      if (ya + 1 < p.y_hi)
        st_chk(dst, (zg * p.GY + (p.oy + ya + 1 - p.gy) % p.GY) * p.GX + xg, p.dst_extent, v.im);
    }
  }
}

template <typename T>
size_t cx_bytes() {
  return sizeof(cx<T>);
}

}  // namespace

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_xfwd(const XFwdParams<T>& p, int nfields, int nthreads, hipStream_t s) {
  const size_t lds = (size_t)(p.ty / 2) * lds_stride(p.NX) * cx_bytes<T>();
  dim3 grid((unsigned)(p.ytiles * p.NZ), (unsigned)nfields);
  hipLaunchKernelGGL(k_xfwd<T>, grid, dim3(nthreads), lds, s, p);
}

template <typename T>
void launch_ypass(const YPassParams<T>& p, int nfields, int nouter, int inverse, int nthreads, hipStream_t s) {
  const size_t lds = (size_t)p.nl * lds_stride(p.n) * cx_bytes<T>();
  dim3 grid((unsigned)(p.utiles * nouter), (unsigned)nfields);
  if (inverse)
    hipLaunchKernelGGL((k_ypass<1, T>), grid, dim3(nthreads), lds, s, p);
  else
    hipLaunchKernelGGL((k_ypass<-1, T>), grid, dim3(nthreads), lds, s, p);
}

template <typename T>
void launch_zpush(const ZPushParams<T>& p, int nthreads, hipStream_t s) {
  const size_t lds = (size_t)11 * lds_stride(p.NZ) * cx_bytes<T>();
  if (lds > 64 * 1024) {
    // Opt in to more than 64 KB of dynamic LDS (the plan checked the device limit).
    static size_t granted = 0;
    if (lds > granted &&
        hipFuncSetAttribute((const void*)k_zpush<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) ==
            hipSuccess)
      granted = lds;
  }
  dim3 grid((unsigned)((i64)p.NXH * p.NY));
  hipLaunchKernelGGL(k_zpush<T>, grid, dim3(nthreads), lds, s, p);
}

template <typename T>
void launch_xinv(const XInvParams<T>& p, int nfields, int nthreads, hipStream_t s) {
  const size_t lds = (size_t)(p.ty / 2) * lds_stride(p.NX) * cx_bytes<T>();
  dim3 grid((unsigned)(p.ytiles * (p.z_hi - p.z_lo)), (unsigned)nfields);
  hipLaunchKernelGGL(k_xinv<T>, grid, dim3(nthreads), lds, s, p);
}

template void launch_xfwd<float>(const XFwdParams<float>&, int, int, hipStream_t);
template void launch_xfwd<double>(const XFwdParams<double>&, int, int, hipStream_t);
template void launch_ypass<float>(const YPassParams<float>&, int, int, int, int, hipStream_t);
template void launch_ypass<double>(const YPassParams<double>&, int, int, int, int, hipStream_t);
template void launch_zpush<float>(const ZPushParams<float>&, int, hipStream_t);
template void launch_zpush<double>(const ZPushParams<double>&, int, hipStream_t);
template void launch_xinv<float>(const XInvParams<float>&, int, int, hipStream_t);
template void launch_xinv<double>(const XInvParams<double>&, int, int, hipStream_t);

}  // namespace psatd
