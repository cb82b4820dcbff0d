// Guard-width surrogate network on the GPU: forward, backward and Adam (gfx950).
//
// The paper calls a model of the number of guard cells n_g required by a local
// solver, as a function of its order, time step and cell size, crucial (Sec.
// 1.4; n_g drives memory and cost, Sec. 2.2) and leaves it open.  This file
// evaluates and trains a 6 -> 64 -> 64 -> 1 network that predicts log10 of the
// local-vs-global truncation error of a run from six features of it:
//
//   x  = (features - in_mean) * in_scale        (per-feature standardisation)
//   h1 = silu(W1 x + b1),  h2 = silu(W2 h1 + b2),  u = W3 h2 + b3
//   prediction = out_mean + out_scale * u
//   loss over a batch of B samples = (1/B) sum (u - (target - out_mean) / out_scale)^2
//
// Weights live twice: an FP32 master copy that Adam updates and a bfloat16
// copy (round to nearest, ties to even) that the forward and backward kernels
// read.  Activations, products and sums are FP32.  The 64-wide layers are far
// too small for matrix-core tiles to pay at these batch sizes, so the products
// are FP32 FMAs on LDS-resident tiles.
//
// Parameter vector (a documented format): W1 (64 x 6, row-major out x in), b1,
// W2 (64 x 64), b2, W3 (64), b3 -- 4673 values.
//
// Gradients are deterministic: each block writes the partial gradient of its
// sample tile, and a second kernel sums the partials in block order.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/psatd.h"
#include "internal.hpp"

namespace {

constexpr int NIN = 6, NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;
static_assert(NPARAM == PSATD_MLP_NPARAM, "parameter count");
constexpr int TS = 32;       // samples per tile (one tile per block)
constexpr int NT = 256;      // threads per block
constexpr int LD = NH + 1;   // padded row length of the LDS activation tiles
constexpr int SB = TS / 16;  // sample rows per thread in the (sample, unit) mappings

struct Norm {
  float in_mean[NIN];
  float in_scale[NIN];
  float out_mean, out_scale;
};

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float -> bfloat16, round to nearest with ties to even; NaN stays a quiet NaN
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu_d(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

struct Tile {
  float w1[NH * NIN], b1[NH], w2[NH * LD], b2[NH], w3[NH], b3;
  float x[TS * NIN], t[TS], valid[TS], dy[TS], lossv[TS];
  float h1[TS * LD], d1[TS * LD], h2[TS * LD], d2[TS * LD];
};

// Stage weights and the tile's (standardised) inputs; samples past the batch
// or with an out-of-range index are masked out (valid = 0, inputs 0).
__device__ void load_tile(Tile& L, const uint16_t* __restrict__ w, const float* __restrict__ X,
                          const float* __restrict__ tgt, int n, const int* __restrict__ idx, int first, int count,
                          const Norm& nm) {
  const int tid = threadIdx.x;
  for (int i = tid; i < NH * NIN; i += NT) L.w1[i] = bf16_to_f32(w[OFF_W1 + i]);
  for (int i = tid; i < NH * NH; i += NT) L.w2[(i >> 6) * LD + (i & 63)] = bf16_to_f32(w[OFF_W2 + i]);
  if (tid < NH) {
    L.b1[tid] = bf16_to_f32(w[OFF_B1 + tid]);
    L.b2[tid] = bf16_to_f32(w[OFF_B2 + tid]);
    L.w3[tid] = bf16_to_f32(w[OFF_W3 + tid]);
  }
  if (tid == 0) L.b3 = bf16_to_f32(w[OFF_B3]);
  if (tid < TS) {
    const int b = first + tid;  // position in the batch
    int s = -1;
    if (b < count) s = idx ? idx[b] : b;
    const bool ok = s >= 0 && s < n;
    L.valid[tid] = ok ? 1.0f : 0.0f;
    for (int k = 0; k < NIN; ++k)
      L.x[tid * NIN + k] = ok ? (X[(size_t)s * NIN + k] - nm.in_mean[k]) * nm.in_scale[k] : 0.0f;
    L.t[tid] = (ok && tgt) ? (tgt[s] - nm.out_mean) / nm.out_scale : 0.0f;
  }
  __syncthreads();
}

// h1, h2 (and silu' of their pre-activations) for the tile; returns u for sample tid < TS in u_out.
__device__ void forward_tile(Tile& L, float* u_out) {
  const int tid = threadIdx.x;
  const int sb = tid >> 4, jb = tid & 15;
#pragma unroll
  for (int b = 0; b < SB; ++b) {
    const int s = sb + 16 * b;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int j = jb + 16 * a;
      float z = L.b1[j];
#pragma unroll
      for (int k = 0; k < NIN; ++k) z = fmaf(L.w1[j * NIN + k], L.x[s * NIN + k], z);
      L.h1[s * LD + j] = silu_f(z);
      L.d1[s * LD + j] = silu_d(z);
    }
  }
  __syncthreads();
  float acc[SB][4];
#pragma unroll
  for (int b = 0; b < SB; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) acc[b][a] = L.b2[jb + 16 * a];
  for (int i = 0; i < NH; ++i) {
    float hv[SB], wv[4];
#pragma unroll
    for (int b = 0; b < SB; ++b) hv[b] = L.h1[(sb + 16 * b) * LD + i];
#pragma unroll
    for (int a = 0; a < 4; ++a) wv[a] = L.w2[(jb + 16 * a) * LD + i];
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int a = 0; a < 4; ++a) acc[b][a] = fmaf(wv[a], hv[b], acc[b][a]);
  }
#pragma unroll
  for (int b = 0; b < SB; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int s = sb + 16 * b, j = jb + 16 * a;
      L.h2[s * LD + j] = silu_f(acc[b][a]);
      L.d2[s * LD + j] = silu_d(acc[b][a]);
    }
  __syncthreads();
  if (tid < TS) {
    float u = L.b3;
    for (int j = 0; j < NH; ++j) u = fmaf(L.w3[j], L.h2[tid * LD + j], u);
    *u_out = u;
  }
}

__global__ void __launch_bounds__(NT) k_mlp_forward(const uint16_t* __restrict__ w, const float* __restrict__ X,
                                                     int n, float* __restrict__ y, Norm nm) {
  __shared__ Tile L;
  const int first = blockIdx.x * TS;
  load_tile(L, w, X, nullptr, n, nullptr, first, n, nm);
  float u = 0.0f;
  forward_tile(L, &u);
  const int tid = threadIdx.x;
  if (tid < TS && first + tid < n) y[first + tid] = nm.out_mean + nm.out_scale * u;
}

// Partial MSE gradient of one tile of the batch (batch positions first .. first+TS-1).
__global__ void __launch_bounds__(NT) k_mlp_grad(const uint16_t* __restrict__ w, const float* __restrict__ X,
                                                  const float* __restrict__ tgt, int n, const int* __restrict__ idx,
                                                  int count, float* __restrict__ part, float* __restrict__ lossp,
                                                  Norm nm) {
  __shared__ Tile L;
  const int tid = threadIdx.x;
  const int first = blockIdx.x * TS;
  load_tile(L, w, X, tgt, n, idx, first, count, nm);
  float u = 0.0f;
  forward_tile(L, &u);
  if (tid < TS) {
    const float r = (u - L.t[tid]) * L.valid[tid];
    L.dy[tid] = 2.0f * r / (float)count;
    L.lossv[tid] = r * r;
  }
  __syncthreads();
  float* g = part + (size_t)blockIdx.x * NPARAM;
  const int sb = tid >> 4, jb = tid & 15;
  // dz2 = dy * W3 * silu'(z2), in place of silu'(z2)
#pragma unroll
  for (int b = 0; b < SB; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int s = sb + 16 * b, j = jb + 16 * a;
      L.d2[s * LD + j] *= L.dy[s] * L.w3[j];
    }
  __syncthreads();
  // dW2[j][i] = sum_s dz2[s][j] h1[s][i]   (thread: j = jb + 16a, i = ib + 16c)
  {
    const int ib = tid >> 4;
    float acc[4][4] = {};
    for (int s = 0; s < TS; ++s) {
      float dv[4], hv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) dv[a] = L.d2[s * LD + jb + 16 * a];
#pragma unroll
      for (int c = 0; c < 4; ++c) hv[c] = L.h1[s * LD + ib + 16 * c];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = fmaf(dv[a], hv[c], acc[a][c]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c) g[OFF_W2 + (jb + 16 * a) * NH + ib + 16 * c] = acc[a][c];
  }
  // dz1[s][i] = silu'(z1[s][i]) * sum_j W2[j][i] dz2[s][j], in place of silu'(z1)
  {
    const int ib = tid & 15;
    float acc[SB][4] = {};
    for (int j = 0; j < NH; ++j) {
      float dv[SB], wv[4];
#pragma unroll
      for (int b = 0; b < SB; ++b) dv[b] = L.d2[(sb + 16 * b) * LD + j];
#pragma unroll
      for (int c = 0; c < 4; ++c) wv[c] = L.w2[j * LD + ib + 16 * c];
#pragma unroll
      for (int b = 0; b < SB; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[b][c] = fmaf(wv[c], dv[b], acc[b][c]);
    }
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int c = 0; c < 4; ++c) L.d1[(sb + 16 * b) * LD + ib + 16 * c] *= acc[b][c];
  }
  __syncthreads();
  // dW1[j][k] = sum_s dz1[s][j] x[s][k]
  for (int o = tid; o < NH * NIN; o += NT) {
    const int j = o / NIN, k = o - j * NIN;
    float acc = 0.0f;
    for (int s = 0; s < TS; ++s) acc = fmaf(L.d1[s * LD + j], L.x[s * NIN + k], acc);
    g[OFF_W1 + o] = acc;
  }
  // biases, W3, and the loss partial
  if (tid < NH) {
    float a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    for (int s = 0; s < TS; ++s) {
      a1 += L.d1[s * LD + tid];
      a2 += L.d2[s * LD + tid];
      a3 = fmaf(L.dy[s], L.h2[s * LD + tid], a3);
    }
    g[OFF_B1 + tid] = a1;
    g[OFF_B2 + tid] = a2;
    g[OFF_W3 + tid] = a3;
  } else if (tid == NH) {
    float a = 0.0f, l = 0.0f;
    for (int s = 0; s < TS; ++s) {
      a += L.dy[s];
      l += L.lossv[s];
    }
    g[OFF_B3] = a;
    lossp[blockIdx.x] = l;
  }
}

// grad[p] = sum over blocks (in block order) of the partials; loss = sum of loss partials / count
__global__ void k_mlp_reduce(const float* __restrict__ part, const float* __restrict__ lossp, int nblk, int count,
                             float* __restrict__ grad, float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NPARAM) {
    float a = 0.0f;
    for (int b = 0; b < nblk; ++b) a += part[(size_t)b * NPARAM + p];
    grad[p] = a;
  } else if (p == NPARAM) {
    float l = 0.0f;
    for (int b = 0; b < nblk; ++b) l += lossp[b];
    *loss = l / (float)count;
  }
}

// One Adam step on the FP32 master weights; refreshes the bfloat16 copy.
__global__ void k_mlp_adam(float* __restrict__ master, uint16_t* __restrict__ wbf, float* __restrict__ m,
                           float* __restrict__ v, const float* __restrict__ grad, float lr, float beta1, float beta2,
                           float eps, float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float g = grad[p];
  const float mm = beta1 * m[p] + (1.0f - beta1) * g;
  const float vv = beta2 * v[p] + (1.0f - beta2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float w = master[p] - lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
  master[p] = w;
  wbf[p] = f32_to_bf16(w);
}

__global__ void k_mlp_round(const float* __restrict__ master, uint16_t* __restrict__ wbf) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NPARAM) wbf[p] = f32_to_bf16(master[p]);
}

__global__ void k_mlp_zero(float* __restrict__ a, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) a[p] = 0.0f;
}

}  // namespace

struct psatd_mlp {
  float* master = nullptr;
  uint16_t* wbf = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  float* loss = nullptr;
  float* part = nullptr;
  float* lossp = nullptr;
  int max_batch = 0;
  long long step = 0;
  Norm nm{};
};

namespace {

using psatd::report_error;

int hip_fail(const char* where) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return report_error(PSATD_EHIP, "%s: %s", where, hipGetErrorString(e));
  return PSATD_OK;
}

void free_mlp(psatd_mlp* p) {
  if (!p) return;
  for (void* q : {(void*)p->master, (void*)p->wbf, (void*)p->m, (void*)p->v, (void*)p->grad, (void*)p->loss,
                  (void*)p->part, (void*)p->lossp})
    if (q) (void)hipFree(q);
  delete p;
}

int nblocks(int n, int per) { return (n + per - 1) / per; }

void enqueue_grad(psatd_mlp* p, const float* X, const float* t, int n, const int* idx, int count, hipStream_t s) {
  const int nb = nblocks(count, TS);
  k_mlp_grad<<<nb, NT, 0, s>>>(p->wbf, X, t, n, idx, count, p->part, p->lossp, p->nm);
  k_mlp_reduce<<<nblocks(NPARAM + 1, 256), 256, 0, s>>>(p->part, p->lossp, nb, count, p->grad, p->loss);
}

void enqueue_adam(psatd_mlp* p, float lr, float beta1, float beta2, float eps, hipStream_t s) {
  ++p->step;
  const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)p->step));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)p->step));
  k_mlp_adam<<<nblocks(NPARAM, 256), 256, 0, s>>>(p->master, p->wbf, p->m, p->v, p->grad, lr, beta1, beta2, eps,
                                                   bc1, bc2);
}

bool adam_args_ok(float lr, float beta1, float beta2, float eps) {
  return std::isfinite(lr) && lr > 0.f && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f &&
         std::isfinite(eps) && eps >= 0.f;
}

}  // namespace

extern "C" {

int psatd_mlp_create(const float* init, const float* in_mean, const float* in_scale, float out_mean,
                     float out_scale, int max_batch, psatd_mlp** out) {
  if (!out) return report_error(PSATD_EINVAL, "psatd_mlp_create: out is NULL");
  *out = nullptr;
  if (!init || !in_mean || !in_scale)
    return report_error(PSATD_EINVAL, "psatd_mlp_create: init, in_mean and in_scale are required");
  if (max_batch < 1 || max_batch > (1 << 24))
    return report_error(PSATD_EINVAL, "psatd_mlp_create: max_batch %d outside [1, 2^24]", max_batch);
  if (!(std::isfinite(out_scale) && out_scale != 0.f) || !std::isfinite(out_mean))
    return report_error(PSATD_EINVAL, "psatd_mlp_create: out_scale must be finite and nonzero");
  psatd_mlp* p = new psatd_mlp;
  p->max_batch = max_batch;
  for (int k = 0; k < NIN; ++k) {
    p->nm.in_mean[k] = in_mean[k];
    p->nm.in_scale[k] = in_scale[k];
  }
  p->nm.out_mean = out_mean;
  p->nm.out_scale = out_scale;
  const size_t pb = sizeof(float) * NPARAM;
  const int nb = nblocks(max_batch, TS);
  if (hipMalloc(&p->master, pb) != hipSuccess || hipMalloc(&p->wbf, sizeof(uint16_t) * NPARAM) != hipSuccess ||
      hipMalloc(&p->m, pb) != hipSuccess || hipMalloc(&p->v, pb) != hipSuccess ||
      hipMalloc(&p->grad, pb) != hipSuccess || hipMalloc(&p->loss, sizeof(float)) != hipSuccess ||
      hipMalloc(&p->part, pb * (size_t)nb) != hipSuccess || hipMalloc(&p->lossp, sizeof(float) * nb) != hipSuccess) {
    (void)hipGetLastError();
    free_mlp(p);
    return report_error(PSATD_ENOMEM, "psatd_mlp_create: device allocation failed");
  }
  const int rc = psatd_mlp_set(p, init);
  if (rc) {
    free_mlp(p);
    return rc;
  }
  *out = p;
  return PSATD_OK;
}

int psatd_mlp_set(psatd_mlp* p, const float* master) {
  if (!p || !master) return report_error(PSATD_EINVAL, "psatd_mlp_set: NULL argument");
  if (hipMemcpy(p->master, master, sizeof(float) * NPARAM, hipMemcpyHostToDevice) != hipSuccess)
    return hip_fail("psatd_mlp_set copy");
  k_mlp_round<<<nblocks(NPARAM, 256), 256>>>(p->master, p->wbf);
  k_mlp_zero<<<nblocks(NPARAM, 256), 256>>>(p->m, NPARAM);
  k_mlp_zero<<<nblocks(NPARAM, 256), 256>>>(p->v, NPARAM);
  p->step = 0;
  if (hipDeviceSynchronize() != hipSuccess) return hip_fail("psatd_mlp_set");
  return hip_fail("psatd_mlp_set");
}

int psatd_mlp_get(const psatd_mlp* p, float* master, unsigned short* bf16) {
  if (!p) return report_error(PSATD_EINVAL, "psatd_mlp_get: NULL plan");
  if (hipDeviceSynchronize() != hipSuccess) return hip_fail("psatd_mlp_get");
  if (master && hipMemcpy(master, p->master, sizeof(float) * NPARAM, hipMemcpyDeviceToHost) != hipSuccess)
    return hip_fail("psatd_mlp_get master");
  if (bf16 && hipMemcpy(bf16, p->wbf, sizeof(uint16_t) * NPARAM, hipMemcpyDeviceToHost) != hipSuccess)
    return hip_fail("psatd_mlp_get bf16");
  return PSATD_OK;
}

int psatd_mlp_predict(const psatd_mlp* p, const float* X, int n, float* y, void* stream) {
  if (!p || (n > 0 && (!X || !y))) return report_error(PSATD_EINVAL, "psatd_mlp_predict: NULL argument");
  if (n < 0) return report_error(PSATD_EINVAL, "psatd_mlp_predict: n = %d", n);
  if (n == 0) return PSATD_OK;
  k_mlp_forward<<<nblocks(n, TS), NT, 0, (hipStream_t)stream>>>(p->wbf, X, n, y, p->nm);
  return hip_fail("psatd_mlp_predict");
}

int psatd_mlp_grad(psatd_mlp* p, const float* X, const float* t, int n, const int* idx, int batch, float* grad,
                   float* loss, void* stream) {
  if (!p || !X || !t) return report_error(PSATD_EINVAL, "psatd_mlp_grad: NULL argument");
  if (n < 1 || batch < 1 || batch > p->max_batch || (!idx && batch > n))
    return report_error(PSATD_EINVAL, "psatd_mlp_grad: n = %d, batch = %d (max %d)", n, batch, p->max_batch);
  hipStream_t s = (hipStream_t)stream;
  enqueue_grad(p, X, t, n, idx, batch, s);
  if (grad) (void)hipMemcpyAsync(grad, p->grad, sizeof(float) * NPARAM, hipMemcpyDeviceToDevice, s);
  if (loss) (void)hipMemcpyAsync(loss, p->loss, sizeof(float), hipMemcpyDeviceToDevice, s);
  return hip_fail("psatd_mlp_grad");
}

int psatd_mlp_adam(psatd_mlp* p, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!p) return report_error(PSATD_EINVAL, "psatd_mlp_adam: NULL plan");
  if (!adam_args_ok(lr, beta1, beta2, eps)) return report_error(PSATD_EINVAL, "psatd_mlp_adam: bad hyperparameters");
  enqueue_adam(p, lr, beta1, beta2, eps, (hipStream_t)stream);
  return hip_fail("psatd_mlp_adam");
}

int psatd_mlp_train(psatd_mlp* p, const float* X, const float* t, int n, const int* idx, int nsteps, int batch,
                    float lr, float beta1, float beta2, float eps, float* loss_hist, void* stream) {
  if (!p || !X || !t) return report_error(PSATD_EINVAL, "psatd_mlp_train: NULL argument");
  if (n < 1 || nsteps < 0 || batch < 1 || batch > p->max_batch || (!idx && batch > n))
    return report_error(PSATD_EINVAL, "psatd_mlp_train: n = %d, nsteps = %d, batch = %d (max %d)", n, nsteps, batch,
                        p->max_batch);
  if (!adam_args_ok(lr, beta1, beta2, eps)) return report_error(PSATD_EINVAL, "psatd_mlp_train: bad hyperparameters");
  hipStream_t s = (hipStream_t)stream;
  for (int k = 0; k < nsteps; ++k) {
    enqueue_grad(p, X, t, n, idx ? idx + (size_t)k * batch : nullptr, batch, s);
    if (loss_hist) (void)hipMemcpyAsync(loss_hist + k, p->loss, sizeof(float), hipMemcpyDeviceToDevice, s);
    enqueue_adam(p, lr, beta1, beta2, eps, s);
  }
  return hip_fail("psatd_mlp_train");
}

void psatd_mlp_destroy(psatd_mlp* p) { free_mlp(p); }

}  // extern "C"
