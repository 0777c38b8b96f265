// FP32 HIP kernels of the learned-start network and their C-ABI entry points.
//
// The network maps a coarse sample of the operator's velocity field
// (2 x h x w) to one start vector on the same grid; it is a stack of 3x3
// dilated convolutions with zero padding, ReLU between layers.  Training
// minimises the fraction of the prediction outside the wanted invariant
// subspace, 1 - ||V^T u||^2 / ||u||^2, with Adam.  The predicted vector is
// resampled bilinearly to the full grid and handed to rks_solve as u0.
// Tensors are dense row-major: activations B x C x H x W, weights
// O x C x 3 x 3, targets B x P x K (P = H W).
#include <hip/hip_runtime.h>

#include "rks.h"

namespace {

__global__ __launch_bounds__(256) void k_conv_fwd(const float* __restrict__ x, const float* __restrict__ w,
                                                  const float* __restrict__ bias, float* __restrict__ y, int B, int C,
                                                  int O, int H, int W, int dil, int relu) {
  const int64_t total = (int64_t)B * O * H * W;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx % W);
    const int i = (int)((idx / W) % H);
    const int o = (int)((idx / ((int64_t)W * H)) % O);
    const int b = (int)(idx / ((int64_t)W * H * O));
    float acc = bias[o];
    for (int c = 0; c < C; ++c) {
      const float* xc = x + ((int64_t)b * C + c) * H * W;
      const float* wc = w + ((int64_t)o * C + c) * 9;
#pragma unroll
      for (int di = 0; di < 3; ++di) {
        const int ii = i + dil * (di - 1);
        if (ii < 0 || ii >= H) continue;
#pragma unroll
        for (int dj = 0; dj < 3; ++dj) {
          const int jj = j + dil * (dj - 1);
          if (jj < 0 || jj >= W) continue;
          acc += wc[di * 3 + dj] * xc[ii * W + jj];
        }
      }
    }
    y[idx] = (relu && acc < 0.f) ? 0.f : acc;
  }
}

// g = dy masked by the layer's ReLU (y > 0) when relu; dx = transposed convolution of g.
__global__ __launch_bounds__(256) void k_conv_bwd_data(const float* __restrict__ dy, const float* __restrict__ y,
                                                       const float* __restrict__ w, float* __restrict__ dx, int B,
                                                       int C, int O, int H, int W, int dil, int relu) {
  const int64_t total = (int64_t)B * C * H * W;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx % W);
    const int i = (int)((idx / W) % H);
    const int c = (int)((idx / ((int64_t)W * H)) % C);
    const int b = (int)(idx / ((int64_t)W * H * C));
    float acc = 0.f;
    for (int o = 0; o < O; ++o) {
      const int64_t base = ((int64_t)b * O + o) * H * W;
      const float* wc = w + ((int64_t)o * C + c) * 9;
#pragma unroll
      for (int di = 0; di < 3; ++di) {
        const int ii = i - dil * (di - 1);
        if (ii < 0 || ii >= H) continue;
#pragma unroll
        for (int dj = 0; dj < 3; ++dj) {
          const int jj = j - dil * (dj - 1);
          if (jj < 0 || jj >= W) continue;
          const int64_t p = base + ii * W + jj;
          float g = dy[p];
          if (relu && !(y[p] > 0.f)) g = 0.f;
          acc += wc[di * 3 + dj] * g;
        }
      }
    }
    dx[idx] = acc;
  }
}

// dw[o, c, tap] = sum_{b, pixel} g[b, o, pixel] x[b, c, pixel + offset(tap)];
// db[o] = sum g[b, o, :].  One block per (o, c); fixed-order block reduction.
__global__ __launch_bounds__(256) void k_conv_bwd_filter(const float* __restrict__ x, const float* __restrict__ dy,
                                                         const float* __restrict__ y, float* __restrict__ dw,
                                                         float* __restrict__ db, int B, int C, int O, int H, int W,
                                                         int dil, int relu) {
  const int o = blockIdx.x / C, c = blockIdx.x % C;
  float acc[10];
#pragma unroll
  for (int t = 0; t < 10; ++t) acc[t] = 0.f;
  const int64_t npix = (int64_t)B * H * W;
  for (int64_t q = threadIdx.x; q < npix; q += blockDim.x) {
    const int b = (int)(q / ((int64_t)H * W));
    const int pix = (int)(q % ((int64_t)H * W));
    const int i = pix / W, j = pix % W;
    const int64_t p = ((int64_t)b * O + o) * H * W + pix;
    float g = dy[p];
    if (relu && !(y[p] > 0.f)) g = 0.f;
    if (g == 0.f) continue;
    const float* xc = x + ((int64_t)b * C + c) * H * W;
#pragma unroll
    for (int di = 0; di < 3; ++di) {
      const int ii = i + dil * (di - 1);
#pragma unroll
      for (int dj = 0; dj < 3; ++dj) {
        const int jj = j + dil * (dj - 1);
        if (ii >= 0 && ii < H && jj >= 0 && jj < W) acc[di * 3 + dj] += g * xc[ii * W + jj];
      }
    }
    acc[9] += g;
  }
  __shared__ float red[10][256];
#pragma unroll
  for (int t = 0; t < 10; ++t) red[t][threadIdx.x] = acc[t];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int t = 0; t < 10; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 9) dw[((int64_t)o * C + c) * 9 + threadIdx.x] = red[threadIdx.x][0];
  if (threadIdx.x == 9 && c == 0) db[o] = red[9][0];
}

// Per sample b: loss[b] = 1 - ||V_b^T u_b||^2/||u_b||^2 and
// du_b = -2 (V_b V_b^T u_b - rho u_b) / ||u_b||^2 / B.  One block per sample.
__global__ __launch_bounds__(256) void k_subspace_loss(const float* __restrict__ u, const float* __restrict__ V,
                                                       float* __restrict__ loss, float* __restrict__ du, int B,
                                                       int P, int K) {
  constexpr int KM = 32;
  const int b = blockIdx.x;
  const float* ub = u + (int64_t)b * P;
  const float* Vb = V + (int64_t)b * P * K;
  __shared__ float red[KM + 1][256];
  __shared__ float pk[KM + 1];
  float acc[KM + 1];
#pragma unroll
  for (int k = 0; k <= KM; ++k) acc[k] = 0.f;
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    const float up = ub[p];
#pragma unroll
    for (int k = 0; k < KM; ++k)
      if (k < K) acc[k] += Vb[(int64_t)p * K + k] * up;
    acc[KM] += up * up;
  }
#pragma unroll
  for (int k = 0; k <= KM; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k <= KM; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if ((int)threadIdx.x <= KM) pk[threadIdx.x] = red[threadIdx.x][0];
  __syncthreads();
  const float uu = pk[KM];
  float pp = 0.f;
  for (int k = 0; k < K; ++k) pp += pk[k] * pk[k];
  const float rho = pp / uu;
  if (threadIdx.x == 0) loss[b] = 1.f - rho;
  const float scale = -2.f / (uu * (float)B);
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    float vp = 0.f;
    for (int k = 0; k < K; ++k) vp += Vb[(int64_t)p * K + k] * pk[k];
    du[(int64_t)b * P + p] = scale * (vp - rho * ub[p]);
  }
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Bilinear resampling with half-pixel centres, clamped to the grid.
__global__ __launch_bounds__(256) void k_upsample(const float* __restrict__ u, int h, int w, double* __restrict__ out,
                                                  int H, int W) {
  const int64_t total = (int64_t)H * W;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int I = (int)(idx / W), J = (int)(idx % W);
    double y = ((double)I + 0.5) * h / H - 0.5;
    double x = ((double)J + 0.5) * w / W - 0.5;
    y = fmin(fmax(y, 0.0), (double)(h - 1));
    x = fmin(fmax(x, 0.0), (double)(w - 1));
    const int y0 = (int)floor(y), x0 = (int)floor(x);
    const int y1 = y0 + 1 < h ? y0 + 1 : h - 1, x1 = x0 + 1 < w ? x0 + 1 : w - 1;
    const double fy = y - y0, fx = x - x0;
    out[idx] = (1.0 - fy) * ((1.0 - fx) * u[y0 * w + x0] + fx * u[y0 * w + x1]) +
               fy * ((1.0 - fx) * u[y1 * w + x0] + fx * u[y1 * w + x1]);
  }
}

int grid_of(int64_t total) {
  int64_t g = (total + 255) / 256;
  if (g > 65535) g = 65535;
  return (int)(g < 1 ? 1 : g);
}

int ok_or_hip() { return hipGetLastError() == hipSuccess ? RKS_OK : RKS_EHIP; }

}  // namespace

extern "C" {

int rks_net_conv3x3_forward(const float* x, const float* w, const float* b, float* y, int32_t B, int32_t Cin,
                            int32_t Cout, int32_t H, int32_t W, int32_t dil, int32_t relu, void* stream) {
  if (!x || !w || !b || !y || B < 1 || Cin < 1 || Cout < 1 || H < 1 || W < 1 || dil < 1) return RKS_EINVAL;
  const int64_t total = (int64_t)B * Cout * H * W;
  k_conv_fwd<<<grid_of(total), 256, 0, (hipStream_t)stream>>>(x, w, b, y, B, Cin, Cout, H, W, dil, relu);
  return ok_or_hip();
}

int rks_net_conv3x3_backward(const float* x, const float* w, const float* y, const float* dy, float* dx, float* dw,
                             float* db, int32_t B, int32_t Cin, int32_t Cout, int32_t H, int32_t W, int32_t dil,
                             int32_t relu, void* stream) {
  if (!x || !w || !dy || !dw || !db || (relu && !y) || B < 1 || Cin < 1 || Cout < 1 || H < 1 || W < 1 || dil < 1)
    return RKS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  k_conv_bwd_filter<<<Cout * Cin, 256, 0, st>>>(x, dy, y, dw, db, B, Cin, Cout, H, W, dil, relu);
  if (dx) {
    const int64_t total = (int64_t)B * Cin * H * W;
    k_conv_bwd_data<<<grid_of(total), 256, 0, st>>>(dy, y, w, dx, B, Cin, Cout, H, W, dil, relu);
  }
  return ok_or_hip();
}

int rks_net_subspace_loss(const float* u, const float* V, float* loss, float* du, int32_t B, int32_t P, int32_t K,
                          void* stream) {
  if (!u || !V || !loss || !du || B < 1 || P < 1 || K < 1 || K > 32) return RKS_EINVAL;
  k_subspace_loss<<<B, 256, 0, (hipStream_t)stream>>>(u, V, loss, du, B, P, K);
  return ok_or_hip();
}

int rks_net_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                 int32_t t, void* stream) {
  if (!w || !g || !m || !v || n < 0 || t < 1) return RKS_EINVAL;
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  k_adam<<<grid_of(n), 256, 0, (hipStream_t)stream>>>(w, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return ok_or_hip();
}

int rks_net_upsample(const float* u, int32_t h, int32_t w, double* out, int32_t H, int32_t W, void* stream) {
  if (!u || !out || h < 1 || w < 1 || H < 1 || W < 1) return RKS_EINVAL;
  k_upsample<<<grid_of((int64_t)H * W), 256, 0, (hipStream_t)stream>>>(u, h, w, out, H, W);
  return ok_or_hip();
}

}  // extern "C"
