// Warm-start surrogate kernels for gfx950: 3x3 dilated convolutions as
// implicit GEMMs on MFMA (bf16 x bf16 -> fp32, v_mfma_f32_16x16x16_bf16),
// their backward passes, masked MSE, Adam, and the feature / target /
// initial-field kernels that connect the network to the lattice solver.
//
// Layouts: activations (B, H, W, C) channels-last, C a multiple of 16;
// weights (Cout, 3, 3, Cin); bf16 values are stored as raw uint16 bits.
// Tap (ky, kx) reads the input at (h + (ky-1) d, w + (kx-1) d), zero outside.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rmrt {
namespace nn {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                           // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float sigmoidf_(float y) { return 1.0f / (1.0f + __expf(-y)); }

enum { EPI_NONE = 0, EPI_SILU = 1, EPI_SILU_GRAD = 2 };

// One wave computes 16 consecutive pixels x all Cout channels (Cout <= 32).
// A[m][k] = input(pixel m shifted by the tap)[channel k], B[k][n] = W[n][tap][k];
// lane l supplies A[l % 16][4 (l / 16) + i] and B[4 (l / 16) + i][l % 16],
// and receives D[4 (l / 16) + i][l % 16], i = 0..3.  Backward-data runs this
// kernel on weights flipped by k_flip.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256)
    k_conv(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w, const float* __restrict__ bias,
           float* __restrict__ y_pre, uint16_t* __restrict__ a_out, const float* __restrict__ aux, int B, int H,
           int W, int dil, int epi) {
  constexpr int NB = COUT / 16;
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * (blockDim.x >> 6)) + (threadIdx.x >> 6);
  const long P = (long)B * H * W;
  const long p0 = (long)wave * 16;
  if (p0 >= P) return;
  const int m = lane & 15, kq = lane >> 4;
  const long pm = p0 + m;                       // pixel supplying row m of A
  const int b = (int)(pm / ((long)H * W));
  const int rem = (int)(pm - (long)b * H * W);
  const int h = rem / W, wq = rem - h * W;
  float4_t acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int ky = tap / 3, kx = tap % 3;
    const int hh = h + (ky - 1) * dil, ww = wq + (kx - 1) * dil;
    const bool inside = (pm < P) && hh >= 0 && hh < H && ww >= 0 && ww < W;
    const uint16_t* xp = x + (((long)b * H + hh) * W + ww) * CIN;
#pragma unroll
    for (int kc = 0; kc < CIN / 16; ++kc) {
      const int c0 = kc * 16 + kq * 4;
      short4_t av = short4_t{0, 0, 0, 0};
      if (inside) av = *(const short4_t*)(xp + c0);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int n = nb * 16 + m;
        const short4_t bv = *(const short4_t*)(w + ((long)n * 9 + tap) * CIN + c0);
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[nb], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long p = p0 + kq * 4 + i;
      const int n = nb * 16 + m;
      if (p >= P) continue;
      float v = acc[nb][i] + (bias ? bias[n] : 0.f);
      if (y_pre) y_pre[p * COUT + n] = v;
      if (epi == EPI_SILU) {
        v = v * sigmoidf_(v);
      } else if (epi == EPI_SILU_GRAD) {
        const float yv = aux[p * COUT + n];
        const float s = sigmoidf_(yv);
        v = v * s * (1.f + yv * (1.f - s));
      }
      if (a_out) a_out[p * COUT + n] = f2bf(v);
    }
  }
}

// wt[ci][ky][kx][co] = w[co][2 - ky][2 - kx][ci]: backward-data as a forward conv
__global__ void k_flip(const uint16_t* __restrict__ w, uint16_t* __restrict__ wt, int Cout, int Cin) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = Cout * 9 * Cin;
  if (i >= n) return;
  const int co = i / (9 * Cin);
  const int r = i - co * 9 * Cin;
  const int tap = r / Cin, ci = r - tap * Cin;
  const int ky = tap / 3, kx = tap % 3;
  wt[((long)ci * 9 + (2 - ky) * 3 + (2 - kx)) * Cout + co] = w[i];
}

// dW[co][tap][ci] partials: one wave per (pixel chunk, tap); A = dY^T (co x pixels),
// B = shifted X (pixels x ci).  Partials are summed by k_wgrad_reduce in fixed order.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256)
    k_wgrad(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dy, float* __restrict__ part, int B, int H,
            int W, int dil, int chunk, int nchunks) {
  constexpr int MB = COUT / 16, NB = CIN / 16;
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * (blockDim.x >> 6)) + (threadIdx.x >> 6);
  if (wave >= nchunks * 9) return;
  const int tap = wave % 9, ck = wave / 9;
  const int ky = tap / 3, kx = tap % 3;
  const long P = (long)B * H * W;
  const int m = lane & 15, kq = lane >> 4;
  float4_t acc[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[a][c] = float4_t{0.f, 0.f, 0.f, 0.f};
  const long pbeg = (long)ck * chunk;
  for (long ps = pbeg; ps < pbeg + chunk && ps < P; ps += 16) {
    short4_t av[MB], bv[NB];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long p = ps + kq * 4 + i;
      bool ok = p < P;
      long src = 0;
      if (ok) {
        const int b = (int)(p / ((long)H * W));
        const int rem = (int)(p - (long)b * H * W);
        const int h = rem / W, wq = rem - h * W;
        const int hh = h + (ky - 1) * dil, ww = wq + (kx - 1) * dil;
        const bool in = hh >= 0 && hh < H && ww >= 0 && ww < W;
        src = (((long)b * H + hh) * W + ww);
#pragma unroll
        for (int a = 0; a < MB; ++a) av[a][i] = (short)dy[p * COUT + a * 16 + m];
#pragma unroll
        for (int c = 0; c < NB; ++c) bv[c][i] = in ? (short)x[src * CIN + c * 16 + m] : (short)0;
      } else {
#pragma unroll
        for (int a = 0; a < MB; ++a) av[a][i] = 0;
#pragma unroll
        for (int c = 0; c < NB; ++c) bv[c][i] = 0;
      }
    }
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int c = 0; c < NB; ++c) acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[c], acc[a][c], 0, 0, 0);
  }
  // D[row = co][col = ci]: lane holds rows 4 kq + i, column m
  float* out = part + ((long)ck * 9 + tap) * COUT * CIN;
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int c = 0; c < NB; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) out[(a * 16 + kq * 4 + i) * CIN + c * 16 + m] = acc[a][c][i];
}

// dw[co][tap][ci] = sum over chunks of part[chunk][tap][co][ci]
__global__ void k_wgrad_reduce(const float* __restrict__ part, float* __restrict__ dw, int Cout, int Cin, int nchunks) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Cout * 9 * Cin) return;
  const int co = i / (9 * Cin);
  const int r = i - co * 9 * Cin;
  const int tap = r / Cin, ci = r - tap * Cin;
  float s = 0.f;
  for (int k = 0; k < nchunks; ++k) s += part[(((long)k * 9 + tap) * Cout + co) * Cin + ci];
  dw[i] = s;
}

// db[co] = sum_p dy[p][co]: per-block partials then a fixed-order final sum
__global__ void k_bgrad_part(const uint16_t* __restrict__ dy, float* __restrict__ part, long P, int Cout) {
  __shared__ float sh[256];
  const int co = threadIdx.x % Cout;
  const int lanes = 256 / Cout;
  const int slot = threadIdx.x / Cout;
  float s = 0.f;
  if (slot < lanes)
    for (long p = (long)blockIdx.x * lanes + slot; p < P; p += (long)gridDim.x * lanes) s += bf2f(dy[p * Cout + co]);
  sh[threadIdx.x] = s;
  __syncthreads();
  if ((int)threadIdx.x < Cout) {
    float t = 0.f;
    for (int k = 0; k < lanes; ++k) t += sh[k * Cout + threadIdx.x];
    part[(long)blockIdx.x * Cout + threadIdx.x] = t;
  }
}
__global__ void k_bgrad_final(const float* __restrict__ part, float* __restrict__ db, int nb, int Cout) {
  const int co = threadIdx.x;
  if (co >= Cout) return;
  float s = 0.f;
  for (int k = 0; k < nb; ++k) s += part[(long)k * Cout + co];
  db[co] = s;
}

// sum of the pixel weights (per-block partials, then k_inv_final)
__global__ void k_wsum(const float* __restrict__ mask, long P, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (long)gridDim.x * blockDim.x) s += mask[p];
  sh[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < (int)blockDim.x; ++k) t += sh[k];
    part[blockIdx.x] = t;
  }
}
__global__ void k_inv_final(const double* __restrict__ part, int nb, float* __restrict__ inv_den) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += part[k];
    inv_den[0] = s > 0.0 ? (float)(1.0 / s) : 0.f;
  }
}

// masked MSE over the first C channels of out (stride Cs): per-block loss
// partials; dout (bf16, stride Cs, zero in the padding channels)
__global__ void k_mse(const float* __restrict__ out, int Cs, const float* __restrict__ tgt, const float* __restrict__ mask,
                      long P, int C, const float* __restrict__ inv_den_p, uint16_t* __restrict__ dout,
                      double* __restrict__ part) {
  __shared__ double sh[256];
  const float inv_den = inv_den_p[0];
  double s = 0.0;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (long)gridDim.x * blockDim.x) {
    const float mk = mask[p];
    for (int c = 0; c < Cs; ++c) {
      float g = 0.f;
      if (c < C) {
        const float dlt = out[p * Cs + c] - tgt[p * C + c];
        s += (double)mk * dlt * dlt;
        g = 2.f * mk * dlt * inv_den;
      }
      dout[p * Cs + c] = f2bf(g);
    }
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < (int)blockDim.x; ++k) t += sh[k];
    part[blockIdx.x] = t;
  }
}
__global__ void k_sum_final(const double* __restrict__ part, int nb, const float* __restrict__ scale,
                            double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += part[k];
    out[0] = s * (double)scale[0];
  }
}

// Adam with bias correction; w32 master weights, optional bf16 copy
__global__ void k_adam(float* __restrict__ w, uint16_t* __restrict__ wbf, const float* __restrict__ g,
                       float* __restrict__ mo, float* __restrict__ vo, long n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float m = b1 * mo[i] + (1.f - b1) * gi;
  const float v = b2 * vo[i] + (1.f - b2) * gi * gi;
  mo[i] = m;
  vo[i] = v;
  const float wi = w[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  w[i] = wi;
  if (wbf) wbf[i] = f2bf(wi);
}

__global__ void k_to_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = f2bf(src[i]);
}

// ---------------------------------------------------------------------------
// Glue between the lattice solver (fine grid, nodes x-fastest, walls at the
// y faces) and the network (coarse grid, k x k blocks, channels-last).
// Coarse pixel (b, i, j): rows i (y), columns j (x).  The Poiseuille prior is
// 4 y (H - y) / H^2 at the physical height y of the cell centre.
// ---------------------------------------------------------------------------
// colfrac[b][x] = solid fraction of column x; gfrac[b] = solid fraction of sample b
__global__ void k_colfrac(const uint8_t* __restrict__ solid, int B, int nx, int ny, float* __restrict__ colfrac) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)B * nx) return;
  const int b = (int)(t / nx), x = (int)(t - (long)b * nx);
  int cnt = 0;
  for (int y = 0; y < ny; ++y) cnt += solid[((long)b * ny + y) * nx + x] ? 1 : 0;
  colfrac[t] = (float)cnt / (float)ny;
}
__global__ void k_gfrac(const float* __restrict__ colfrac, int B, int nx, float* __restrict__ gfrac) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double s = 0.0;
  for (int x = 0; x < nx; ++x) s += colfrac[(long)b * nx + x];
  gfrac[b] = (float)(s / nx);
}

// features: ch0 = solid fraction of the block, ch1 = prior, ch2 = Re / re_scale,
// ch3 = solid fraction of the block's columns over the full height (local
// constriction), ch4 = solid fraction of the whole channel, ch5.. = 0
__global__ void k_features(const uint8_t* __restrict__ solid, const float* __restrict__ re, int B, int nx, int ny, int k,
                           float dy, float re_scale, const float* __restrict__ colfrac, const float* __restrict__ gfrac,
                           uint16_t* __restrict__ x0, int Cs) {
  const int hc = ny / k, wc = nx / k;
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (long)B * hc * wc) return;
  const int b = (int)(p / ((long)hc * wc));
  const int r = (int)(p - (long)b * hc * wc);
  const int i = r / wc, j = r - i * wc;
  int cnt = 0;
  for (int a = 0; a < k; ++a)
    for (int c = 0; c < k; ++c) cnt += solid[(long)b * nx * ny + (long)(i * k + a) * nx + (j * k + c)] ? 1 : 0;
  const float Hh = ny * dy;
  const float y = (i * k + 0.5f * k) * dy;
  const float prior = 4.f * y * (Hh - y) / (Hh * Hh);
  float col = 0.f;
  for (int c = 0; c < k; ++c) col += colfrac[(long)b * nx + j * k + c];
  col /= (float)k;
  for (int c = 0; c < Cs; ++c) {
    float v = 0.f;
    if (c == 0) v = (float)cnt / (float)(k * k);
    if (c == 1) v = prior;
    if (c == 2) v = re[b] / re_scale;
    if (c == 3) v = col;
    if (c == 4) v = gfrac[b];
    x0[p * Cs + c] = f2bf(v);
  }
}

// targets: fluid means over the block of (u / Ut - prior(y_node)), v / Ut,
// (rho - 1) rho_scale; weight = fluid fraction of the block
__global__ void k_targets(const double* __restrict__ rho, const double* __restrict__ u, const uint8_t* __restrict__ solid,
                          int B, int nx, int ny, int k, float dy, float Ut, float rho_scale, float* __restrict__ tgt,
                          float* __restrict__ wgt) {
  const int hc = ny / k, wc = nx / k;
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (long)B * hc * wc) return;
  const int b = (int)(p / ((long)hc * wc));
  const int r = (int)(p - (long)b * hc * wc);
  const int i = r / wc, j = r - i * wc;
  const long N = (long)nx * ny;
  const float Hh = ny * dy;
  double s0 = 0, s1 = 0, s2 = 0;
  int cnt = 0;
  for (int a = 0; a < k; ++a)
    for (int c = 0; c < k; ++c) {
      const int yy = i * k + a, xx = j * k + c;
      const long n = (long)yy * nx + xx;
      if (solid[b * N + n]) continue;
      const float y = (yy + 0.5f) * dy;
      const float prior = 4.f * y * (Hh - y) / (Hh * Hh);
      s0 += u[(long)b * 2 * N + n] / Ut - prior;
      s1 += u[(long)b * 2 * N + N + n] / Ut;
      s2 += (rho[b * N + n] - 1.0) * rho_scale;
      ++cnt;
    }
  const double inv = cnt ? 1.0 / cnt : 0.0;
  tgt[p * 3 + 0] = (float)(s0 * inv);
  tgt[p * 3 + 1] = (float)(s1 * inv);
  tgt[p * 3 + 2] = (float)(s2 * inv);
  wgt[p] = (float)cnt / (float)(k * k);
}

// initial fields on the fine grid from the coarse prediction (bilinear,
// positions (node + 1/2) / k - 1/2 in coarse units, clamped):
// u = Ut (prior(y) + o0), v = Ut o1, rho = 1 + o2 / rho_scale; zero velocity in solids
__global__ void k_warm_fields(const float* __restrict__ out, int Cs, int B, int nx, int ny, int k, float dy, float Ut,
                              float rho_scale, const uint8_t* __restrict__ solid, double* __restrict__ rho,
                              double* __restrict__ u) {
  const int hc = ny / k, wc = nx / k;
  const long N = (long)nx * ny;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)B * N) return;
  const int b = (int)(t / N);
  const long n = t - (long)b * N;
  const int yy = (int)(n / nx), xx = (int)(n - (long)yy * nx);
  float py = (yy + 0.5f) / k - 0.5f, px = (xx + 0.5f) / k - 0.5f;
  py = fminf(fmaxf(py, 0.f), (float)(hc - 1));
  px = fminf(fmaxf(px, 0.f), (float)(wc - 1));
  const int i0 = (int)floorf(py), j0 = (int)floorf(px);
  const int i1 = min(i0 + 1, hc - 1), j1 = min(j0 + 1, wc - 1);
  const float fy = py - i0, fx = px - j0;
  float o[3];
  for (int c = 0; c < 3; ++c) {
    const float* base = out + (long)b * hc * wc * Cs;
    const float v00 = base[((long)i0 * wc + j0) * Cs + c], v01 = base[((long)i0 * wc + j1) * Cs + c];
    const float v10 = base[((long)i1 * wc + j0) * Cs + c], v11 = base[((long)i1 * wc + j1) * Cs + c];
    o[c] = (v00 * (1 - fx) + v01 * fx) * (1 - fy) + (v10 * (1 - fx) + v11 * fx) * fy;
  }
  const float Hh = ny * dy;
  const float y = (yy + 0.5f) * dy;
  const float prior = 4.f * y * (Hh - y) / (Hh * Hh);
  const bool s = solid && solid[b * N + n];
  rho[b * N + n] = 1.0 + (double)o[2] / rho_scale;
  u[(long)b * 2 * N + n] = s ? 0.0 : (double)(Ut * (prior + o[0]));
  u[(long)b * 2 * N + N + n] = s ? 0.0 : (double)(Ut * o[1]);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t launch_conv(const uint16_t* x, const uint16_t* w, const float* bias, float* y_pre, uint16_t* a_out,
                       const float* aux, int B, int H, int W, int Cin, int Cout, int dil, int epi, hipStream_t s) {
  const long P = (long)B * H * W;
  const long waves = (P + 15) / 16;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
#define CONV_CASE(CI, CO)                                                                                      \
  if (Cin == CI && Cout == CO) {                                                                               \
    hipLaunchKernelGGL((k_conv<CI, CO>), dim3(blocks), dim3(256), 0, s, x, w, bias, y_pre, a_out, aux, B, H, W, \
                       dil, epi);                                                                              \
    return hipGetLastError();                                                                                  \
  }
  CONV_CASE(16, 16) CONV_CASE(16, 32) CONV_CASE(32, 16) CONV_CASE(32, 32)
#undef CONV_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_flip(const uint16_t* w, uint16_t* wt, int Cout, int Cin, hipStream_t s) {
  const int n = Cout * 9 * Cin;
  hipLaunchKernelGGL(k_flip, dim3((n + 255) / 256), dim3(256), 0, s, w, wt, Cout, Cin);
  return hipGetLastError();
}

size_t wgrad_partial_floats(long P, int Cin, int Cout, int chunk) {
  const long nchunks = (P + chunk - 1) / chunk;
  return (size_t)nchunks * 9 * Cin * Cout;
}

hipError_t launch_wgrad(const uint16_t* x, const uint16_t* dy, int B, int H, int W, int Cin, int Cout, int dil, float* dw,
                        float* db, float* part, size_t part_floats, hipStream_t s) {
  const long P = (long)B * H * W;
  const int chunk = 1024;
  const int nchunks = (int)((P + chunk - 1) / chunk);
  if (wgrad_partial_floats(P, Cin, Cout, chunk) > part_floats) return hipErrorInvalidValue;
  if ((size_t)1024 * Cout > part_floats) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((nchunks * 9 + 3) / 4);
#define WG_CASE(CI, CO)                                                                                              \
  if (Cin == CI && Cout == CO) {                                                                                     \
    hipLaunchKernelGGL((k_wgrad<CI, CO>), dim3(blocks), dim3(256), 0, s, x, dy, part, B, H, W, dil, chunk, nchunks); \
  } else
  WG_CASE(16, 16) WG_CASE(16, 32) WG_CASE(32, 16) WG_CASE(32, 32) { return hipErrorInvalidValue; }
#undef WG_CASE
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = Cout * 9 * Cin;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((n + 255) / 256), dim3(256), 0, s, part, dw, Cout, Cin, nchunks);
  e = hipGetLastError();
  if (e != hipSuccess || !db) return e;
  // bias gradient reuses the (already consumed) partial buffer
  const int nb = 1024;
  hipLaunchKernelGGL(k_bgrad_part, dim3(nb), dim3(256), 0, s, dy, part, P, Cout);
  hipLaunchKernelGGL(k_bgrad_final, dim3(1), dim3(64), 0, s, part, db, nb, Cout);
  return hipGetLastError();
}

// scratch: >= 2 * kMseBlocks doubles; loss: one double (device); inv_den: one float (device)
constexpr int kMseBlocks = 512;
hipError_t launch_mse(const float* out, int Cs, const float* tgt, const float* mask, long P, int C, uint16_t* dout,
                      double* scratch, float* inv_den, double* loss, hipStream_t s) {
  const int nb = kMseBlocks;
  hipLaunchKernelGGL(k_wsum, dim3(nb), dim3(256), 0, s, mask, P, scratch);
  hipLaunchKernelGGL(k_inv_final, dim3(1), dim3(64), 0, s, scratch, nb, inv_den);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, out, Cs, tgt, mask, P, C, inv_den, dout, scratch + nb);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(64), 0, s, scratch + nb, nb, inv_den, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, uint16_t* wbf, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, wbf, g, m, v, n, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* src, uint16_t* dst, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

// scratch: B * (nx + 1) floats
hipError_t launch_features(const uint8_t* solid, const float* re, int B, int nx, int ny, int k, float dy, float re_scale,
                           uint16_t* x0, int Cs, float* scratch, hipStream_t s) {
  const long P = (long)B * (ny / k) * (nx / k);
  float* colfrac = scratch;
  float* gfrac = scratch + (long)B * nx;
  hipLaunchKernelGGL(k_colfrac, dim3((unsigned)(((long)B * nx + 255) / 256)), dim3(256), 0, s, solid, B, nx, ny, colfrac);
  hipLaunchKernelGGL(k_gfrac, dim3((B + 63) / 64), dim3(64), 0, s, colfrac, B, nx, gfrac);
  hipLaunchKernelGGL(k_features, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, solid, re, B, nx, ny, k, dy,
                     re_scale, colfrac, gfrac, x0, Cs);
  return hipGetLastError();
}

hipError_t launch_targets(const double* rho, const double* u, const uint8_t* solid, int B, int nx, int ny, int k,
                          float dy, float Ut, float rho_scale, float* tgt, float* wgt, hipStream_t s) {
  const long P = (long)B * (ny / k) * (nx / k);
  hipLaunchKernelGGL(k_targets, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, rho, u, solid, B, nx, ny, k, dy,
                     Ut, rho_scale, tgt, wgt);
  return hipGetLastError();
}

hipError_t launch_warm_fields(const float* out, int Cs, int B, int nx, int ny, int k, float dy, float Ut,
                              float rho_scale, const uint8_t* solid, double* rho, double* u, hipStream_t s) {
  const long n = (long)B * nx * ny;
  hipLaunchKernelGGL(k_warm_fields, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, Cs, B, nx, ny, k, dy, Ut,
                     rho_scale, solid, rho, u);
  return hipGetLastError();
}

}  // namespace nn
}  // namespace rmrt
