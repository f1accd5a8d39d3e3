// Learned partitioner (not part of the paper): an FP32 CDF model
// 1 -> 64 -> 64 -> 1 (ReLU hidden layers) trained on the method's own sorted
// sample, used to propose the root level's zone splitters.  All arithmetic
// runs on the FP32 vector units.
//
// Parameter layout (4353 floats): W1[64], b1[64], W2[64][64] (row = output
// unit), b2[64], W3[64], b3.  Loss: mean squared error.  Optimiser: Adam.
// Inputs: x = log-linear transform of the key (one unit per binary order of
// magnitude, linear inside it), rescaled to [0, 1] over the sample; target
// y = (rank + 0.5) / N.  Batches: step s uses samples j*stride + (s mod
// stride), j < batch, stride = N / batch.
#include <hip/hip_runtime.h>

#include <vector>

#include "block_sort.hpp"
#include "launch.hpp"

namespace dts {

constexpr int NP = 4353;
constexpr int OW1 = 0, OB1 = 64, OW2 = 128, OB2 = 128 + 4096, OW3 = 128 + 4096 + 64, OB3 = 128 + 4096 + 128;

__device__ inline double u01(uint64_t h, uint64_t i) {
  return (double)(mix64(h + (i + 1) * GOLD) >> 11) * (1.0 / 9007199254740992.0);
}

// Deterministic initialisation: per hidden unit of layer 1 a kink in [0, 1),
// slope magnitude sqrt(6) (0.5 + 0.5 u), random sign; W2, W3 uniform in
// +-sqrt(6/64); b2 = 0, b3 = 0.5.  Computed in double, stored as float.
__global__ void k_mlp_init(float* p, uint64_t seed) {
  const uint64_t h = mix64(mix64(seed + GOLD) ^ 0x4D4C50ull);
  const double s6 = 2.449489742783178;       // sqrt(6)
  const double s664 = 0.30618621784789724;   // sqrt(6/64)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NP; i += gridDim.x * blockDim.x) {
    float v = 0.0f;
    if (i < OB1) {
      const double a = u01(h, 3ull * i);
      const double mag = s6 * (0.5 + 0.5 * u01(h, 3ull * i + 1));
      const double sg = u01(h, 3ull * i + 2) < 0.5 ? -1.0 : 1.0;
      v = (float)(sg * mag);
    } else if (i < OW2) {
      const int j = i - OB1;
      const int iw = OW1 + j;
      const double a = u01(h, 3ull * iw);
      const double mag = s6 * (0.5 + 0.5 * u01(h, 3ull * iw + 1));
      const double sg = u01(h, 3ull * iw + 2) < 0.5 ? -1.0 : 1.0;
      v = (float)(-(sg * mag) * a);
    } else if (i < OB2) {
      v = (float)((2.0 * u01(h, 3ull * i) - 1.0) * s664);
    } else if (i < OW3) {
      v = 0.0f;
    } else if (i < OB3) {
      v = (float)((2.0 * u01(h, 3ull * i) - 1.0) * s664);
    } else {
      v = 0.5f;
    }
    p[i] = v;
  }
}

template <typename K>
__device__ inline double loglinear(K k, int kb) {
  if (k == 0) return 0.0;
  const int e = bit_length(k) - 1;
  const K p = (K)1 << e;
  const double frac = (double)(k - p) / (double)p;
  return ((double)e + 1.0 + frac) / (double)(kb + 1);
}

// x, y from the sorted sample keys.
template <typename K>
__global__ void k_mlp_data(const K* sk, uint32_t n, int kb, float* x, float* y) {
  const double t0 = loglinear<K>(sk[0], kb);
  const double span = loglinear<K>(sk[n - 1], kb) - t0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double t = loglinear<K>(sk[i], kb);
    x[i] = span > 0 ? (float)((t - t0) / span) : 0.0f;
    y[i] = (float)(((double)i + 0.5) / (double)n);
  }
}

// Forward + backward for GS samples per workgroup; writes this workgroup's
// partial gradient (and partial loss at index NP) to part[blockIdx.x].
// Samples: j = blockIdx.x * GS + s < batch; data index j*stride + off
// (stride 0 = contiguous).  The mean is over `batch`.
//
// The three 64-wide products of a step (Z2 = H1 W2^T, dW2 = dZ2^T H1,
// dH1 = dZ2 W2) run as register tiles: thread t owns ZR sample rows from
// ZR*(t/16) (4 unit rows from 4*(t/16) for dW2) and 4 columns from 4*(t%16)
// and streams the shared dimension from LDS (rows padded to 65 floats against
// bank conflicts).  Every sum over samples is taken in sample order, so
// results are deterministic.
constexpr int GS = 64;     // samples per gradient workgroup
constexpr int GTH = 256;   // threads per gradient workgroup
constexpr int LP = 65;     // padded LDS row
constexpr int ZR = GS / 16;  // sample rows per thread in the (sample x unit) products

__global__ __launch_bounds__(GTH) void k_mlp_grad(const float* __restrict__ p, const float* __restrict__ x,
                                                  const float* __restrict__ y, uint32_t batch, uint32_t stride,
                                                  uint32_t off, float* __restrict__ part) {
  __shared__ float P[NP];
  __shared__ float W2s[64 * LP];  // W2 rows (output unit o), padded
  __shared__ float H1[GS * LP];   // h1[s][i]
  __shared__ float Z2[GS * LP];   // z2[s][o], later dz1[s][i]
  __shared__ float DZ[GS * LP];   // dz2[s][o]
  __shared__ float XS[GS], D[GS], ERR2[GS];
  const int t = threadIdx.x;
  for (int i = t; i < NP; i += GTH) P[i] = p[i];
  __syncthreads();
  for (int e = t; e < 4096; e += GTH) W2s[(e >> 6) * LP + (e & 63)] = P[OW2 + e];
  if (t < GS) {
    const uint32_t j = blockIdx.x * GS + t;
    const uint32_t di = stride ? j * stride + off : j;
    XS[t] = j < batch ? x[di] : 0.0f;
  }
  __syncthreads();
  for (int e = t; e < GS * 64; e += GTH) {
    const int sm = e >> 6, i = e & 63;
    H1[sm * LP + i] = fmaxf(fmaf(P[OW1 + i], XS[sm], P[OB1 + i]), 0.0f);
  }
  __syncthreads();
  const int c0 = (t % 16) * 4;
  const int zr0 = (t / 16) * ZR;  // first sample row of this thread
  const int r0 = (t / 16) * 4;    // first unit row of this thread (dW2)
  // Z2[s][o] = b2[o] + sum_i W2[o][i] h1[s][i]
  {
    float acc[ZR][4];
#pragma unroll
    for (int a = 0; a < ZR; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = P[OB2 + c0 + b];
    for (int i = 0; i < 64; ++i) {
      float hv[ZR], wv[4];
#pragma unroll
      for (int a = 0; a < ZR; ++a) hv[a] = H1[(zr0 + a) * LP + i];
#pragma unroll
      for (int b = 0; b < 4; ++b) wv[b] = W2s[(c0 + b) * LP + i];
#pragma unroll
      for (int a = 0; a < ZR; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(wv[b], hv[a], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < ZR; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) Z2[(zr0 + a) * LP + c0 + b] = acc[a][b];
  }
  __syncthreads();
  // output, error and d = dLoss/dyhat per sample
  if (t < GS) {
    const uint32_t j = blockIdx.x * GS + t;
    const uint32_t di = stride ? j * stride + off : j;
    float yh = P[OB3];  // one thread per sample
    for (int o = 0; o < 64; ++o) yh = fmaf(P[OW3 + o], fmaxf(Z2[t * LP + o], 0.0f), yh);
    const float err = j < batch ? yh - y[di] : 0.0f;
    D[t] = 2.0f * err / (float)batch;
    ERR2[t] = err * err / (float)batch;
  }
  __syncthreads();
  for (int e = t; e < GS * 64; e += GTH) {
    const int sm = e >> 6, o = e & 63;
    DZ[sm * LP + o] = Z2[sm * LP + o] > 0.0f ? D[sm] * P[OW3 + o] : 0.0f;
  }
  float* out = part + (size_t)blockIdx.x * (NP + 1);
  if (t < 64) {
    // dW3[o] = sum_s d_s relu(z2[s][o])
    float s3 = 0.0f;
    for (int sm = 0; sm < GS; ++sm) s3 = fmaf(D[sm], fmaxf(Z2[sm * LP + t], 0.0f), s3);
    out[OW3 + t] = s3;
  } else if (t == 64) {
    float db3 = 0.0f, ls = 0.0f;
    for (int sm = 0; sm < GS; ++sm) {
      db3 += D[sm];
      ls += ERR2[sm];
    }
    out[OB3] = db3;
    out[NP] = ls;
  }
  __syncthreads();
  // dW2[o][i] = sum_s dz2[s][o] h1[s][i]; db2[o] = sum_s dz2[s][o]
  {
    float acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = 0.0f;
    for (int sm = 0; sm < GS; ++sm) {
      float dv[4], hv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) dv[a] = DZ[sm * LP + r0 + a];
#pragma unroll
      for (int b = 0; b < 4; ++b) hv[b] = H1[sm * LP + c0 + b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(dv[a], hv[b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) out[OW2 + (r0 + a) * 64 + c0 + b] = acc[a][b];
  }
  if (t < 64) {
    float sb = 0.0f;
    for (int sm = 0; sm < GS; ++sm) sb += DZ[sm * LP + t];
    out[OB2 + t] = sb;
  }
  // dz1[s][i] = (h1[s][i] > 0) * sum_o W2[o][i] dz2[s][o]  (into Z2's space)
  {
    float acc[ZR][4];
#pragma unroll
    for (int a = 0; a < ZR; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = 0.0f;
    for (int o = 0; o < 64; ++o) {
      float dv[ZR], wv[4];
#pragma unroll
      for (int a = 0; a < ZR; ++a) dv[a] = DZ[(zr0 + a) * LP + o];
#pragma unroll
      for (int b = 0; b < 4; ++b) wv[b] = W2s[o * LP + c0 + b];
#pragma unroll
      for (int a = 0; a < ZR; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(wv[b], dv[a], acc[a][b]);
    }
    __syncthreads();  // every thread is done reading Z2 (dW3 above)
#pragma unroll
    for (int a = 0; a < ZR; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        Z2[(zr0 + a) * LP + c0 + b] = H1[(zr0 + a) * LP + c0 + b] > 0.0f ? acc[a][b] : 0.0f;
  }
  __syncthreads();
  // dW1[i] = sum_s dz1[s][i] x_s; db1[i] = sum_s dz1[s][i]
  if (t < 64) {
    float s1 = 0.0f;
    for (int sm = 0; sm < GS; ++sm) s1 = fmaf(Z2[sm * LP + t], XS[sm], s1);
    out[OW1 + t] = s1;
  } else if (t < 128) {
    const int i = t - 64;
    float sb = 0.0f;
    for (int sm = 0; sm < GS; ++sm) sb += Z2[sm * LP + i];
    out[OB1 + i] = sb;
  }
}

// Sum the partial gradients in workgroup order (deterministic).  adam = 0:
// write the gradient and loss; adam = 1: Adam update of p, m, v at step
// `step` (1-based) and record the loss.
__global__ void k_mlp_reduce(const float* __restrict__ part, uint32_t nwg, float* p, float* m, float* v,
                             float* grad, float* loss_out, int adam, int step, float lr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > NP) return;
  float g = 0.0f;
  for (uint32_t w = 0; w < nwg; ++w) g += part[(size_t)w * (NP + 1) + i];
  if (i == NP) {
    if (loss_out) *loss_out = g;
    return;
  }
  if (!adam) {
    grad[i] = g;
    return;
  }
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float c1 = 1.0f - powf(b1, (float)step);
  const float c2 = 1.0f - powf(b2, (float)step);
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ p, const float* __restrict__ x,
                                                     uint32_t n, float* __restrict__ pred) {
  __shared__ float P[NP];
  for (int i = threadIdx.x; i < NP; i += 256) P[i] = p[i];
  __syncthreads();
  const uint32_t j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const float xs = x[j];
  float h1[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) h1[i] = fmaxf(fmaf(P[OW1 + i], xs, P[OB1 + i]), 0.0f);
  float yh = P[OB3];
#pragma unroll 4
  for (int o = 0; o < 64; ++o) {
    float s = P[OB2 + o];
#pragma unroll
    for (int i = 0; i < 64; ++i) s = fmaf(P[OW2 + o * 64 + i], h1[i], s);
    yh = fmaf(P[OW3 + o], fmaxf(s, 0.0f), yh);
  }
  pred[j] = yh;
}

// ------------------------------------------------------------ launchers
struct MlpBufs {
  float* p;
  float* m;
  float* v;
  float* part;
  uint32_t part_wg;  // capacity in workgroups
};

int mlp_loss_grad(const float* p, const float* x, const float* y, uint32_t n, float* grad, float* loss, float* part,
                  hipStream_t s) {
  const uint32_t nwg = (n + GS - 1) / GS;
  hipLaunchKernelGGL(k_mlp_grad, dim3(nwg), dim3(GTH), 0, s, p, x, y, n, 0u, 0u, part);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((NP + 1 + 255) / 256), dim3(256), 0, s, part, nwg, (float*)nullptr,
                     (float*)nullptr, (float*)nullptr, grad, loss, 0, 0, 0.0f);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

void mlp_forward(const float* p, const float* x, uint32_t n, float* pred, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_mlp_forward, dim3((n + 255) / 256), dim3(256), 0, s, p, x, n, pred);
}

// Full training loop: init, then `steps` Adam steps on strided batches.
void mlp_train(const float* x, const float* y, uint32_t n, uint64_t seed, int steps, uint32_t batch, float lr,
               float* p, float* m, float* v, float* part, float* losses, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_init, dim3(18), dim3(256), 0, s, p, seed);
  (void)hipMemsetAsync(m, 0, sizeof(float) * NP, s);
  (void)hipMemsetAsync(v, 0, sizeof(float) * NP, s);
  const uint32_t stride = n / batch;
  const uint32_t nwg = (batch + GS - 1) / GS;
  for (int st = 0; st < steps; ++st) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(nwg), dim3(GTH), 0, s, (const float*)p, x, y, batch, stride,
                       (uint32_t)(st % stride), part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NP + 1 + 255) / 256), dim3(256), 0, s, (const float*)part, nwg, p, m, v,
                       (float*)nullptr, losses ? losses + st : (float*)nullptr, 1, st + 1, lr);
  }
}

template <typename K>
void mlp_data(const K* sk, uint32_t n, int kb, float* x, float* y, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_data<K>, dim3((n + 255) / 256), dim3(256), 0, s, sk, n, kb, x, y);
}
template void mlp_data<uint64_t>(const uint64_t*, uint32_t, int, float*, float*, hipStream_t);
template void mlp_data<uint32_t>(const uint32_t*, uint32_t, int, float*, float*, hipStream_t);

}  // namespace dts

// ------------------------------------------------------------------ C ABI
#include "../../include/dtsort.h"

namespace {
struct TmpF {
  std::vector<void*> ptrs;
  ~TmpF() {
    for (void* q : ptrs) (void)hipFree(q);
  }
  float* get(size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(float) * (n ? n : 1)) != hipSuccess) return nullptr;
    ptrs.push_back(q);
    return (float*)q;
  }
};
}  // namespace

extern "C" {

int dtsort_mlp_loss_grad(const float* params, const float* x, const float* y, size_t n, float* grad, float* loss,
                         void* stream) {
  if (!params || !x || !y || !grad || !loss || n == 0 || n >= (1u << 31)) return DTSORT_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  TmpF tmp;
  const size_t nwg = (n + dts::GS - 1) / dts::GS;
  float* part = tmp.get(nwg * (dts::NP + 1));
  if (!part) return DTSORT_ENOMEM;
  if (dts::mlp_loss_grad(params, x, y, (uint32_t)n, grad, loss, part, s)) return DTSORT_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? DTSORT_OK : DTSORT_EHIP;
}

int dtsort_mlp_forward(const float* params, const float* x, size_t n, float* pred, void* stream) {
  if (!params || !x || !pred || n >= (1u << 31)) return DTSORT_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  dts::mlp_forward(params, x, (uint32_t)n, pred, s);
  if (hipGetLastError() != hipSuccess) return DTSORT_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? DTSORT_OK : DTSORT_EHIP;
}

int dtsort_mlp_train_u64(const uint64_t* sorted_keys, size_t n, uint64_t seed, int steps, int batch, float lr,
                         float* params, float* losses, void* stream) {
  if (!sorted_keys || !params || n < 2 || n >= (1u << 31) || steps < 0 || batch <= 0 || (size_t)batch > n || !(lr > 0))
    return DTSORT_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  TmpF tmp;
  float* x = tmp.get(n);
  float* y = tmp.get(n);
  float* m = tmp.get(dts::NP);
  float* v = tmp.get(dts::NP);
  float* part = tmp.get(((size_t)batch + dts::GS - 1) / dts::GS * (dts::NP + 1));
  if (!x || !y || !m || !v || !part) return DTSORT_ENOMEM;
  dts::mlp_data<uint64_t>(sorted_keys, (uint32_t)n, 64, x, y, s);
  dts::mlp_train(x, y, (uint32_t)n, seed, steps, (uint32_t)batch, lr, params, m, v, part, losses, s);
  if (hipGetLastError() != hipSuccess) return DTSORT_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? DTSORT_OK : DTSORT_EHIP;
}

}  // extern "C"

// ====================================================================
// Learned root plan: training sample, splitters, balance judge, tables.
// ====================================================================
namespace dts {

// Sample keys at counter-based random positions (the same generator as the
// sampling step, with its own stream tag).
template <typename K>
__global__ void k_draw(const K* keys, uint64_t n, uint64_t seed, uint32_t tag, uint32_t count, K* out) {
  const uint64_t sb = sample_base(seed, 0, tag);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const uint64_t r = mix64(sb + (uint64_t)(i + 1) * GOLD);
    out[i] = keys[__umul64hi(r, n)];
  }
}

// Splitters from the model: running maximum of the predictions over the
// sorted sample, then for every zone boundary b/Z the first sample key whose
// monotone prediction reaches it (one past the largest key if none does),
// made non-decreasing.  One workgroup.
template <typename K>
__global__ __launch_bounds__(1024) void k_splitters(const K* sk, const float* pred, uint32_t n, uint32_t zones,
                                                    float* mono, uint64_t* spl) {
  __shared__ float wmax[16];
  __shared__ float carry;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  if (threadIdx.x == 0) carry = -INFINITY;
  __syncthreads();
  for (uint32_t b0 = 0; b0 < n; b0 += 1024) {
    const uint32_t i = b0 + threadIdx.x;
    float x = i < n ? pred[i] : -INFINITY;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const float y = __shfl_up(x, o, WAVE);
      if (lane >= o) x = fmaxf(x, y);
    }
    if (lane == WAVE - 1) wmax[wv] = x;
    __syncthreads();
    float pre = carry;
    for (int w = 0; w < wv; ++w) pre = fmaxf(pre, wmax[w]);
    x = fmaxf(x, pre);
    if (i < n) mono[i] = x;
    __syncthreads();
    if (threadIdx.x == 1023) carry = x;
    __syncthreads();
  }
  const uint64_t top = (uint64_t)(K)~(K)0;
  for (uint32_t b = threadIdx.x + 1; b < zones; b += 1024) {
    const float q = (float)b / (float)zones;
    uint32_t lo = 0, m = n;
    while (m > 0) {
      const uint32_t half = m >> 1;
      if (mono[lo + half] < q) {
        lo += half + 1;
        m -= half + 1;
      } else {
        m = half;
      }
    }
    uint64_t s;
    if (lo < n) {
      s = (uint64_t)sk[lo];
    } else {
      const uint64_t mx = (uint64_t)sk[n - 1];
      s = mx < top ? mx + 1 : top;
    }
    spl[b - 1] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t last = 0;
    for (uint32_t b = 0; b + 1 < zones; ++b) {
      last = spl[b] > last ? spl[b] : last;
      spl[b] = last;
    }
  }
}

// Predicted work below a root plan, in record passes: a zone of s records
// costs s x (1 + the distribution levels it still needs), a zone above the
// base-case cutoff needing log2(s / cutoff) / g levels of g-bit digits (each
// level divides a subproblem by about 2^g; counted fractionally, so that
// zones just either side of the cutoff cost about the same, as the sampled
// sizes are only estimates).  counts are held-out light keys per zone,
// scaled by `scale` records each.
__device__ inline float zone_levels(float sz, float cutoff, int g) {
  return sz > cutoff ? log2f(sz / cutoff) / (float)g : 0.f;
}

__device__ inline float zones_cost(const uint32_t* counts, uint32_t zones, float scale, float cutoff, int g) {
  float tot = 0.f;
  for (uint32_t z = 0; z < zones; ++z) {
    const float sz = (float)counts[z] * scale;
    tot += sz * (1.f + zone_levels(sz, cutoff, g));
  }
  return tot;
}

// Judge of the learned partitioner.  On a held-out sample of the task's
// keys (heavy keys excluded: both plans share the sampling detector's), it
// predicts the work each root plan leaves (zones_cost) for the digit plan
// already in the slot (the sampling step's; keys above its sampled range
// form one more zone) and, when splitters are given, for the model's Z
// zones.  Without splitters it only records the digit plan's cost and the
// cost of an ideal Z-zone split, and whether training could pay
// (digit > train_margin x ideal).  With splitters the model's zones are used
// when their cost is below use_margin x the digit plan's (or always with
// `force`); then the task's light-id table is rewritten for splitter zones
// and the task marked.  Balance errors (largest zone / ideal) are recorded
// too.  One workgroup.
template <typename K>
__global__ __launch_bounds__(1024) void k_judge(Task* task, uint8_t* tab, const K* held, uint32_t nh_keys,
                                                const uint64_t* spl_in, uint32_t Z, JudgeParams jp, LearnedInfo* info,
                                                const float* losses, int steps) {
  __shared__ uint32_t cd[(1 << GMAX) + 1], cl[1 << GMAX];
  __shared__ uint32_t hz[1 << (GMAX - 1)];
  __shared__ K H[1 << (GMAX - 1)];
  __shared__ K SPL[1 << GMAX];
  __shared__ uint32_t light_cnt;
  __shared__ int use;
  Task t = *task;
  const bool full = spl_in != nullptr;
  const SlotLayout sl = slot_layout(t.gamma, true);
  uint8_t* slot = tab + t.tab_off;
  uint32_t* gL = (uint32_t*)(slot + sl.light);
  const uint64_t* gH = (const uint64_t*)(slot + sl.heavy);
  uint64_t* gS = (uint64_t*)(slot + sl.spl);
  const uint32_t zd = 1u << t.w;
  for (uint32_t i = threadIdx.x; i <= zd; i += 1024) cd[i] = 0;
  for (uint32_t i = threadIdx.x; i < Z; i += 1024) cl[i] = 0;
  for (uint32_t i = threadIdx.x; i < t.n_heavy; i += 1024) H[i] = (K)gH[i];
  if (full)
    for (uint32_t i = threadIdx.x; i + 1 < Z; i += 1024) SPL[i] = (K)spl_in[i];
  if (threadIdx.x == 0) light_cnt = 0;
  __syncthreads();
  const K mhi = mask_below<K>(t.hi);
  for (uint32_t i = threadIdx.x; i < nh_keys; i += 1024) {
    const K k = held[i];
    uint32_t lo = 0, m = t.n_heavy;
    while (m > 0) {
      const uint32_t half = m >> 1;
      if (H[lo + half] < k) {
        lo += half + 1;
        m -= half + 1;
      } else {
        m = half;
      }
    }
    if (lo < t.n_heavy && H[lo] == k) continue;
    atomicAdd(&light_cnt, 1u);
    const K low = k & mhi;
    if (t.top >= t.hi || shr<K>(low, t.top) == 0)
      atomicAdd(&cd[(uint32_t)(shr<K>(low, t.shift) & (K)(zd - 1u))], 1u);
    else
      atomicAdd(&cd[zd], 1u);  // above the sampled range: the overflow bucket
    if (full) {
      uint32_t a = 0, n2 = Z - 1;
      while (n2 > 0) {
        const uint32_t half = n2 >> 1;
        if (SPL[a + half] <= k) {
          a += half + 1;
          n2 -= half + 1;
        } else {
          n2 = half;
        }
      }
      atomicAdd(&cl[a], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const float lc = (float)max(light_cnt, 1u);
    uint32_t md = 0;
    for (uint32_t z = 0; z < zd; ++z) md = max(md, cd[z]);
    info->bal_digit = (float)md / (lc / (float)zd);
    info->light_held = light_cnt;
    info->cost_digit = zones_cost(cd, zd + 1, jp.scale, jp.cutoff, jp.g_digit);
    // ideal: the light keys spread evenly over Z zones
    const float each = (float)light_cnt / (float)Z * jp.scale;
    info->cost_ideal = (float)light_cnt * jp.scale * (1.f + zone_levels(each, jp.cutoff, jp.g_learned));
    use = 0;
    if (!full) {
      info->trained = jp.force || info->cost_digit > jp.train_margin * info->cost_ideal;
      info->use_learned = 0;
      info->bal_learned = 0.f;
      info->cost_learned = 0.f;
      info->final_loss = 0.f;
    } else {
      uint32_t ml = 0;
      for (uint32_t z = 0; z < Z; ++z) ml = max(ml, cl[z]);
      info->bal_learned = (float)ml / (lc / (float)Z);
      info->cost_learned = zones_cost(cl, Z, jp.scale, jp.cutoff, jp.g_learned);
      info->trained = 1;
      info->final_loss = steps > 0 ? losses[steps - 1] : 0.0f;
      use = jp.force || info->cost_learned < jp.use_margin * info->cost_digit;
      info->use_learned = use;
    }
  }
  __syncthreads();
  if (!use) return;
  // zones of the heavy keys under the splitters, then light ids
  for (uint32_t i = threadIdx.x; i < t.n_heavy; i += 1024) {
    const K k = H[i];
    uint32_t a = 0, n2 = Z - 1;
    while (n2 > 0) {
      const uint32_t half = n2 >> 1;
      if (SPL[a + half] <= k) {
        a += half + 1;
        n2 -= half + 1;
      } else {
        n2 = half;
      }
    }
    hz[i] = a;
  }
  for (uint32_t i = threadIdx.x; i + 1 < Z; i += 1024) gS[i] = (uint64_t)SPL[i];
  __syncthreads();
  for (uint32_t z = threadIdx.x; z <= Z; z += 1024) {
    uint32_t lo = 0, m = t.n_heavy;
    while (m > 0) {
      const uint32_t half = m >> 1;
      if (hz[lo + half] < z) {
        lo += half + 1;
        m -= half + 1;
      } else {
        m = half;
      }
    }
    gL[z] = z + lo;
  }
  if (threadIdx.x == 0) {
    t.flags = (uint8_t)((t.flags & ~TF_SPLIT) | TF_LEARNED);
    t.w = (uint8_t)(31 - __builtin_clz(Z));
    t.shift = 0;
    t.top = t.hi;
    t.n_buckets = (uint16_t)(Z + t.n_heavy + 1);
    *task = t;
  }
}

template <typename K>
void learned_kernels_draw(const K* keys, uint64_t n, uint64_t seed, uint32_t tag, uint32_t count, K* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_draw<K>, dim3((count + 255) / 256), dim3(256), 0, s, keys, n, seed, tag, count, out);
}
template <typename K>
void learned_kernels_split(const K* sk, const float* pred, uint32_t n, uint32_t zones, float* mono, uint64_t* spl,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_splitters<K>, dim3(1), dim3(1024), 0, s, sk, pred, n, zones, mono, spl);
}
template <typename K>
void learned_kernels_judge(Task* task, uint8_t* tab, const K* held, uint32_t nh, const uint64_t* spl, uint32_t zones,
                           const JudgeParams& jp, LearnedInfo* info, const float* losses, int steps, hipStream_t s) {
  hipLaunchKernelGGL(k_judge<K>, dim3(1), dim3(1024), 0, s, task, tab, held, nh, spl, zones, jp, info, losses, steps);
}
#define DTS_INST(K)                                                                                           \
  template void learned_kernels_draw<K>(const K*, uint64_t, uint64_t, uint32_t, uint32_t, K*, hipStream_t);   \
  template void learned_kernels_split<K>(const K*, const float*, uint32_t, uint32_t, float*, uint64_t*,      \
                                         hipStream_t);                                                       \
  template void learned_kernels_judge<K>(Task*, uint8_t*, const K*, uint32_t, const uint64_t*, uint32_t,     \
                                         const JudgeParams&, LearnedInfo*, const float*, int, hipStream_t);
DTS_INST(uint32_t)
DTS_INST(uint64_t)
#undef DTS_INST

}  // namespace dts
