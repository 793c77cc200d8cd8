// Kernels of the convolutional warm-start network: 3x3 / 1x1 convolutions as
// implicit GEMMs on bf16 matrix cores (gfx950's v_mfma_f32_16x16x32_bf16) with FP32
// accumulation, their weight gradients, and the element-wise layers (ReLU,
// 2x2 average pooling, nearest 2x upsampling with channel concatenation, mean
// squared loss, Adam on FP32 master weights).
//
// Activations are FP32 in memory, [B][H][W][C] (channels fastest); a
// convolution rounds its operands to bf16 (nearest, ties to even) as it stages
// them in LDS.  Weights of a layer with kernel size KS are kept as bf16
// copies Wb[co][k] with k = tap * Ci + ci, tap = di * KS + dj, and, for the
// data gradient, WT[ci][k'] with k' = (KS^2 - 1 - tap) * Co + co (taps
// flipped, channels swapped): the data gradient of a stride-1 zero-padded
// correlation is the correlation of the output gradient with WT.  Both are
// output-channel major (k contiguous), so a weight tile row is one run.
#include <cmath>

#include "internal.hpp"

namespace lsop {

typedef short nn_s4 __attribute__((ext_vector_type(4)));
typedef float nn_f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// Tile 64 (rows) x 64 (columns) per workgroup of four waves (each 32 x 32 =
// 2 x 2 MFMA 16x16 tiles); K staged 32 at a time, LDS rows of NN_SK bf16
// (k contiguous, so each lane's eight k values are one or two reads).
// MFMA 16x16x32 bf16: lane l supplies A[l % 16][8 (l / 16) .. + 7] and
// B[8 (l / 16) .. + 7][l % 16] (both operands take the same k positions, so the
// product does not depend on how the matrix core orders k); register r of the
// result is row 4 (l / 16) + r, column l % 16.
constexpr int NN_T = 64, NN_K = 32, NN_SK = NN_K + 4;

typedef __bf16 nn_bf8 __attribute__((ext_vector_type(8)));

// eight consecutive bf16 of an LDS row: one 16-byte read where rows are 16-byte aligned, else two 8-byte reads
template <int SK>
__device__ __forceinline__ nn_bf8 nn_ld8(const unsigned short* p) {
  if constexpr (SK % 8 == 0) {
    return *reinterpret_cast<const nn_bf8*>(p);
  } else {
    const nn_s4 lo = *reinterpret_cast<const nn_s4*>(p), hi = *reinterpret_cast<const nn_s4*>(p + 4);
    typedef short nn_s8 __attribute__((ext_vector_type(8)));
    const nn_s8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_bit_cast(nn_bf8, v);
  }
}

template <int SK = NN_SK>
__device__ __forceinline__ void nn_mma_stage(const unsigned short* sA, const unsigned short* sB, int wm, int wn, int l,
                                             nn_f4 (&acc)[2][2]) {
  static_assert(NN_K == 32, "one 16x16x32 step per stage");
  nn_bf8 a[2], b[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) a[i] = nn_ld8<SK>(&sA[(wm + i * 16 + (l & 15)) * SK + 8 * (l >> 4)]);
#pragma unroll
  for (int j = 0; j < 2; ++j) b[j] = nn_ld8<SK>(&sB[(wn + j * 16 + (l & 15)) * SK + 8 * (l >> 4)]);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
}

// Y[p][n] = act(bias[n] + sum_k A[p][k] Wb[k][n]) with A the implicit im2col of
// X: A[p][k] = X[b][y + di - R][x + dj - R][c] (zero outside the image),
// k = (di KS + dj) C + c, R = KS / 2, p = (b H + y) W + x.
template <int KS>
__global__ __launch_bounds__(256) void k_conv_fwd(const float* __restrict__ X, int C,
                                                  const unsigned short* __restrict__ Wb, int N,
                                                  const float* __restrict__ bias, float* __restrict__ Y, int B, int H,
                                                  int W, int relu) {
  __shared__ unsigned short sA[NN_T * NN_SK];
  __shared__ unsigned short sB[NN_T * NN_SK];
  const int P = B * H * W, K = KS * KS * C;
  const int p0 = blockIdx.x * NN_T, n0 = blockIdx.y * NN_T;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  nn_f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = nn_f4{0.f, 0.f, 0.f, 0.f};
  const int ap = threadIdx.x >> 2, ak = (threadIdx.x & 3) * 8;  // A loader: pixel, 8 consecutive k
  const int pix = p0 + ap;
  const bool pin = pix < P;
  const int pb = pin ? pix / (H * W) : 0, prem = pin ? pix % (H * W) : 0;
  const int py = prem / W, px = prem % W;
  const int bk = threadIdx.x >> 3, bn = (threadIdx.x & 7) * 8;  // B loader: k, 8 consecutive n
  for (int k0 = 0; k0 < K; k0 += NN_K) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k0 + ak + q;
      float v = 0.f;
      if (pin && k < K) {
        const int tap = k / C, c = k - tap * C;
        const int yy = py + tap / KS - KS / 2, xx = px + tap % KS - KS / 2;
        if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = X[(((size_t)pb * H + yy) * W + xx) * C + c];
      }
      sA[ap * NN_SK + ak + q] = to_bf16(v);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k0 + bk, n = n0 + bn + q;
      sB[(bn + q) * NN_SK + bk] = (k < K && n < N) ? Wb[(size_t)n * K + k] : (unsigned short)0;
    }
    __syncthreads();
    nn_mma_stage(sA, sB, wm, wn, l, acc);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = p0 + wm + i * 16 + 4 * (l >> 4) + r;
        const int n = n0 + wn + j * 16 + (l & 15);
        if (p < P && n < N) {
          float v = acc[i][j][r] + (bias ? bias[n] : 0.f);
          if (relu) v = fmaxf(v, 0.f);
          Y[(size_t)p * N + n] = v;
        }
      }
}

// k_conv_fwd for C % 8 == 0 (so K % 8 == 0, and 8 consecutive k share one
// tap): each thread moves 8 consecutive k of one pixel (two float4 loads, one
// 16-byte bf16 LDS write; one index division per stage) and 8 consecutive k
// of one output channel's weights; the next stage is loaded into registers
// while the current one is multiplied.  X and Wb 16-byte aligned.
constexpr int NN_SKV = NN_K + 8;  // bf16 per LDS row: 16-byte aligned rows, conflict-free MFMA operand reads

__device__ __forceinline__ unsigned nn_pack2(float lo, float hi) {
  return (unsigned)to_bf16(lo) | ((unsigned)to_bf16(hi) << 16);
}

template <int KS>
__global__ __launch_bounds__(256) void k_conv_fwd_v(const float* __restrict__ X, int C,
                                                    const unsigned short* __restrict__ Wb, int N,
                                                    const float* __restrict__ bias, float* __restrict__ Y, int B,
                                                    int H, int W, int relu) {
  __shared__ __align__(16) unsigned short sA[NN_T * NN_SKV];
  __shared__ __align__(16) unsigned short sB[NN_T * NN_SKV];
  const int P = B * H * W, K = KS * KS * C;
  const int p0 = blockIdx.x * NN_T, n0 = blockIdx.y * NN_T;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  nn_f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = nn_f4{0.f, 0.f, 0.f, 0.f};
  const int row = threadIdx.x >> 2, ak = (threadIdx.x & 3) * 8;  // pixel (A) / output channel (B), 8 k
  const int pix = p0 + row;
  const bool pin = pix < P;
  const int pb = pin ? pix / (H * W) : 0, prem = pin ? pix % (H * W) : 0;
  const int py = prem / W, px = prem % W;
  const unsigned short* wrow = (n0 + row < N) ? Wb + (size_t)(n0 + row) * K : nullptr;
  float4 xa, xb;
  uint4 wv;
  auto load = [&](int k0) {
    const int k = k0 + ak;
    xa = make_float4(0.f, 0.f, 0.f, 0.f);
    xb = xa;
    if (pin && k < K) {
      const int tap = k / C, c = k - tap * C;
      const int yy = py + tap / KS - KS / 2, xx = px + tap % KS - KS / 2;
      if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
        const float4* src = reinterpret_cast<const float4*>(X + (((size_t)pb * H + yy) * W + xx) * C + c);
        xa = src[0];
        xb = src[1];
      }
    }
    wv = (wrow && k < K) ? *reinterpret_cast<const uint4*>(wrow + k) : make_uint4(0u, 0u, 0u, 0u);
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += NN_K) {
    *reinterpret_cast<uint4*>(&sA[row * NN_SKV + ak]) =
        make_uint4(nn_pack2(xa.x, xa.y), nn_pack2(xa.z, xa.w), nn_pack2(xb.x, xb.y), nn_pack2(xb.z, xb.w));
    *reinterpret_cast<uint4*>(&sB[row * NN_SKV + ak]) = wv;
    __syncthreads();
    if (k0 + NN_K < K) load(k0 + NN_K);
    nn_mma_stage<NN_SKV>(sA, sB, wm, wn, l, acc);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = p0 + wm + i * 16 + 4 * (l >> 4) + r;
        const int n = n0 + wn + j * 16 + (l & 15);
        if (p < P && n < N) {
          float v = acc[i][j][r] + (bias ? bias[n] : 0.f);
          if (relu) v = fmaxf(v, 0.f);
          Y[(size_t)p * N + n] = v;
        }
      }
}

// dW[k][n] += sum_p A[p][k] dY[p][n] over the pixels [z pchunk, (z + 1) pchunk)
// (A the implicit im2col of X as in k_conv_fwd); FP32 atomic accumulation.
template <int KS>
__global__ __launch_bounds__(256) void k_conv_wgrad(const float* __restrict__ X, int C, const float* __restrict__ dY,
                                                    int N, float* __restrict__ dW, int B, int H, int W, int pchunk) {
  __shared__ unsigned short sA[NN_T * NN_SK];  // [k row][pixel]
  __shared__ unsigned short sB[NN_T * NN_SK];  // [n][pixel]
  const int P = B * H * W, K = KS * KS * C;
  const int k0 = blockIdx.x * NN_T, n0 = blockIdx.y * NN_T;
  const int pbeg = blockIdx.z * pchunk, pend = min(P, pbeg + pchunk);
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  nn_f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = nn_f4{0.f, 0.f, 0.f, 0.f};
  const int lr = threadIdx.x >> 2, lp = (threadIdx.x & 3) * 8;  // loader: row (k or n), 8 consecutive pixels
  const int kr = k0 + lr;
  const bool kin = kr < K;
  const int tap = kin ? kr / C : 0, cc = kin ? kr - tap * C : 0;
  const int dy = tap / KS - KS / 2, dx = tap % KS - KS / 2;
  const int nr = n0 + lr;
  for (int q0 = pbeg; q0 < pend; q0 += NN_K) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int p = q0 + lp + q;
      float va = 0.f, vb = 0.f;
      if (p < pend) {
        const int b = p / (H * W), rem = p % (H * W), y = rem / W + dy, x = rem % W + dx;
        if (kin && y >= 0 && y < H && x >= 0 && x < W) va = X[(((size_t)b * H + y) * W + x) * C + cc];
        if (nr < N) vb = dY[(size_t)p * N + nr];
      }
      sA[lr * NN_SK + lp + q] = to_bf16(va);
      sB[lr * NN_SK + lp + q] = to_bf16(vb);
    }
    __syncthreads();
    nn_mma_stage(sA, sB, wm, wn, l, acc);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = k0 + wm + i * 16 + 4 * (l >> 4) + r;
        const int n = n0 + wn + j * 16 + (l & 15);
        if (k < K && n < N) atomicAdd(&dW[(size_t)k * N + n], acc[i][j][r]);
      }
}

// k_conv_wgrad for C % 8 == 0 and N % 8 == 0: each thread loads, per
// 32-pixel stage, 8 consecutive k (one tap, 8 channels) and 8 consecutive n of
// one pixel as float4 pairs (one index division per stage) and scatters them
// into the pixel-contiguous LDS rows; the next stage is loaded into registers
// while the current one is multiplied.  X and dY 16-byte aligned.
template <int KS>
__global__ __launch_bounds__(256) void k_conv_wgrad_v(const float* __restrict__ X, int C,
                                                      const float* __restrict__ dY, int N, float* __restrict__ dW,
                                                      int B, int H, int W, int pchunk) {
  __shared__ unsigned short sA[NN_T * NN_SK];  // [k row][pixel]
  __shared__ unsigned short sB[NN_T * NN_SK];  // [n][pixel]
  const int P = B * H * W, K = KS * KS * C;
  const int k0 = blockIdx.x * NN_T, n0 = blockIdx.y * NN_T;
  const int pbeg = blockIdx.z * pchunk, pend = min(P, pbeg + pchunk);
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  nn_f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = nn_f4{0.f, 0.f, 0.f, 0.f};
  const int q = threadIdx.x >> 3, c8 = (threadIdx.x & 7) * 8;  // pixel of the stage, 8 consecutive k / n
  const int kr = k0 + c8, nr = n0 + c8;
  const bool kin = kr < K, nin = nr < N;
  const int tap = kin ? kr / C : 0, cc = kin ? kr - tap * C : 0;
  const int dy = tap / KS - KS / 2, dx = tap % KS - KS / 2;
  float4 xa, xb, ga, gb;
  auto load = [&](int q0) {
    const int p = q0 + q;
    xa = make_float4(0.f, 0.f, 0.f, 0.f);
    xb = xa;
    ga = xa;
    gb = xa;
    if (p < pend) {
      const int b = p / (H * W), rem = p % (H * W), y = rem / W + dy, x = rem % W + dx;
      if (kin && y >= 0 && y < H && x >= 0 && x < W) {
        const float4* src = reinterpret_cast<const float4*>(X + (((size_t)b * H + y) * W + x) * C + cc);
        xa = src[0];
        xb = src[1];
      }
      if (nin) {
        const float4* g = reinterpret_cast<const float4*>(dY + (size_t)p * N + nr);
        ga = g[0];
        gb = g[1];
      }
    }
  };
  load(pbeg);
  for (int q0 = pbeg; q0 < pend; q0 += NN_K) {
    const float xv[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
    const float gv[8] = {ga.x, ga.y, ga.z, ga.w, gb.x, gb.y, gb.z, gb.w};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      sA[(c8 + j) * NN_SK + q] = to_bf16(xv[j]);
      sB[(c8 + j) * NN_SK + q] = to_bf16(gv[j]);
    }
    __syncthreads();
    if (q0 + NN_K < pend) load(q0 + NN_K);
    nn_mma_stage(sA, sB, wm, wn, l, acc);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = k0 + wm + i * 16 + 4 * (l >> 4) + r;
        const int n = n0 + wn + j * 16 + (l & 15);
        if (k < K && n < N) atomicAdd(&dW[(size_t)k * N + n], acc[i][j][r]);
      }
}

// db[n] += sum over the pixels [blockIdx.x pchunk, ...) of dY[p][n], N <= 256: the block's first
// T = (256 / N) N threads sweep the chunk as one flat array with stride T, so thread t always meets column
// t % N; the per-thread sums are then reduced per column in LDS (one atomic per column and block).
__global__ __launch_bounds__(256) void k_colsum_flat(const float* __restrict__ dY, int P, int N, int pchunk,
                                                     float* __restrict__ db) {
  __shared__ float red[256];
  const int T = (256 / N) * N, t = threadIdx.x;
  const int pbeg = blockIdx.x * pchunk, pend = min(P, pbeg + pchunk);
  float s = 0.f;
  if (t < T && pbeg < pend) {
    const size_t end = (size_t)pend * N;
    for (size_t i = (size_t)pbeg * N + t; i < end; i += T) s += dY[i];
  }
  red[t] = s;
  __syncthreads();
  if (t < N) {
    float v = 0.f;
    for (int m = t; m < T; m += N) v += red[m];
    atomicAdd(&db[t], v);
  }
}

// db[n] += sum over a pixel chunk of dY[p][n] (any N; one thread per column)
__global__ void k_colsum(const float* __restrict__ dY, int P, int N, int pchunk, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int pbeg = blockIdx.y * pchunk, pend = min(P, pbeg + pchunk);
  float s = 0.f;
  for (int p = pbeg; p < pend; ++p) s += dY[(size_t)p * N + n];
  atomicAdd(&db[n], s);
}

// out[i] = scale * z[stride i] (z: standard normal draws)
__global__ void k_scale_copy(float* __restrict__ out, const float* __restrict__ z, size_t n, int stride,
                             float scale) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    out[k] = scale * z[k * stride];
}

// g = g * (y > 0)
__global__ void k_relu_bwd(float* __restrict__ g, const float* __restrict__ y, size_t n) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    if (!(y[k] > 0.f)) g[k] = 0.f;
}

// y[b][i][j][c] = mean of the 2x2 block of x (x: [B][2h][2w][C])
__global__ void k_avgpool2(const float* __restrict__ x, float* __restrict__ y, int B, int h, int w, int C) {
  const size_t total = (size_t)B * h * w * C;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(k % C);
    size_t t = k / C;
    const int j = (int)(t % w);
    t /= w;
    const int i = (int)(t % h);
    const int b = (int)(t / h);
    const size_t W2 = 2 * (size_t)w, base = (((size_t)b * 2 * h + 2 * i) * W2 + 2 * j) * C + c;
    y[k] = 0.25f * (x[base] + x[base + C] + x[base + W2 * C] + x[base + W2 * C + C]);
  }
}

// dx[b][y][x][c] = dy[b][y / 2][x / 2][c] / 4 + (add ? add[b][y][x][c] : 0)  (dx: [B][2h][2w][C])
__global__ void k_avgpool2_bwd(const float* __restrict__ dy, const float* __restrict__ add, float* __restrict__ dx,
                               int B, int h, int w, int C) {
  const size_t total = (size_t)B * 4 * h * w * C;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(k % C);
    size_t t = k / C;
    const int x = (int)(t % (2 * w));
    t /= 2 * w;
    const int y = (int)(t % (2 * h));
    const int b = (int)(t / (2 * h));
    const float v = 0.25f * dy[(((size_t)b * h + y / 2) * w + x / 2) * C + c];
    dx[k] = add ? v + add[k] : v;
  }
}

// out[b][y][x][:] = [lo[b][y / 2][x / 2][0 .. Cu), skip[b][y][x][0 .. Cs)]  (out at 2h x 2w)
__global__ void k_upcat(const float* __restrict__ lo, const float* __restrict__ skip, float* __restrict__ out, int B,
                        int h, int w, int Cu, int Cs) {
  const int Ct = Cu + Cs;
  const size_t total = (size_t)B * 4 * h * w * Ct;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(k % Ct);
    const size_t pix = k / Ct;
    const int x = (int)(pix % (2 * w));
    const size_t t = pix / (2 * w);
    const int y = (int)(t % (2 * h));
    const int b = (int)(t / (2 * h));
    out[k] = c < Cu ? lo[(((size_t)b * h + y / 2) * w + x / 2) * Cu + c] : skip[pix * Cs + (c - Cu)];
  }
}

// dlo = 2x2 sums of the first Cu channels of dcat; dskip = its last Cs channels
__global__ void k_upcat_bwd(const float* __restrict__ dcat, float* __restrict__ dlo, float* __restrict__ dskip, int B,
                            int h, int w, int Cu, int Cs) {
  const int Ct = Cu + Cs;
  const size_t nlo = (size_t)B * h * w * Cu, nsk = (size_t)B * 4 * h * w * Cs;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < nlo + nsk; k += (size_t)gridDim.x * blockDim.x) {
    if (k < nlo) {
      const int c = (int)(k % Cu);
      size_t t = k / Cu;
      const int j = (int)(t % w);
      t /= w;
      const int i = (int)(t % h);
      const int b = (int)(t / h);
      const size_t W2 = 2 * (size_t)w, p = ((size_t)b * 2 * h + 2 * i) * W2 + 2 * j;
      dlo[k] = dcat[p * Ct + c] + dcat[(p + 1) * Ct + c] + dcat[(p + W2) * Ct + c] + dcat[(p + W2 + 1) * Ct + c];
    } else {
      const size_t q = k - nlo;
      dskip[q] = dcat[(q / Cs) * Ct + Cu + q % Cs];
    }
  }
}

// loss += sum (out - t)^2 / n (double accumulator), dout = 2 (out - t) / n
__global__ void k_mse(const float* __restrict__ out, const float* __restrict__ t, float* __restrict__ dout, size_t n,
                      double* __restrict__ loss) {
  double s = 0.0;
  const float inv = 1.f / (float)n;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const float d = out[k] - t[k];
    dout[k] = 2.f * d * inv;
    s += (double)d * (double)d;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, (red[0] + red[1] + red[2] + red[3]) / (double)n);
}

// Adam (Kingma & Ba, Algorithm 1) on FP32 master weights: m, v moments, bias-corrected step.  The decay
// complements 1 - beta and the bias corrections 1 - beta^t arrive precomputed in FP64 and rounded once:
// 1 - beta2^t formed in FP32 from beta2 = 0.999 loses about 5e-5 of its value to cancellation.
__global__ void k_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M, float* __restrict__ V,
                       size_t n, float lr, float b1, float omb1, float b2, float omb2, float eps, float c1, float c2) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const float g = G[k];
    const float m = b1 * M[k] + omb1 * g;
    const float v = b2 * V[k] + omb2 * g * g;
    M[k] = m;
    V[k] = v;
    P[k] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
  }
}

// bf16 copies of one layer's weights: Wb[k][co] and WT[(KS^2 - 1 - tap) Co + co][ci] from W (FP32 [KS^2 Ci][Co])
__global__ void k_weights_bf16(const float* __restrict__ Wf, int KS, int Ci, int Co, unsigned short* __restrict__ Wb,
                               unsigned short* __restrict__ WT) {
  const int taps = KS * KS;
  const size_t total = (size_t)taps * Ci * Co;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x) {
    const int co = (int)(k % Co);
    const size_t row = k / Co;
    const int ci = (int)(row % Ci), tap = (int)(row / Ci);
    const unsigned short h = to_bf16(Wf[k]);
    Wb[(size_t)co * taps * Ci + row] = h;                                          // [co][tap Ci + ci]
    WT[(size_t)ci * taps * Co + (size_t)(taps - 1 - tap) * Co + co] = h;          // [ci][flipped tap Co + co]
  }
}

// Network input channels per cell from an operator's state and incident
// fields: [c / c0 - 1, Re psi0 / s_v, Im psi0 / s_v, k0 h], with
// c / c0 = (1 + chi c0^2 / omega^2)^(-1/2) from chi = omega^2 (1/c^2 - 1/c0^2)
// and s_v the RMS of incident field v over the grid.
template <typename T>
__global__ void k_pack_inputs(const double* __restrict__ chi, const Cx<T>* __restrict__ psi0,
                              const double* __restrict__ norm2, float* __restrict__ out, size_t n, double c0w2,
                              float k0h, float* __restrict__ scale) {
  const int v = blockIdx.y;
  const double s = sqrt(norm2[v] / (double)n);
  const double inv = s > 0 ? 1.0 / s : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) scale[v] = (float)s;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const double cr = 1.0 / sqrt(1.0 + chi[k] * c0w2);
    const Cx<T> p = psi0[(size_t)v * n + k];
    float* o = out + ((size_t)v * n + k) * 4;
    o[0] = (float)(cr - 1.0);
    o[1] = (float)(p.re * inv);
    o[2] = (float)(p.im * inv);
    o[3] = k0h;
  }
}

// psi = psi0 + s_v (y_re + i y_im) (network output y: [v][n][2])
template <typename T>
__global__ void k_unpack_output(const Cx<T>* __restrict__ psi0, const float* __restrict__ y,
                                const float* __restrict__ scale, Cx<T>* __restrict__ psi, size_t n) {
  const int v = blockIdx.y;
  const float s = scale[v];
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const size_t i = (size_t)v * n + k;
    const Cx<T> p = psi0[i];
    psi[i] = Cx<T>{p.re + (T)(s * y[2 * i]), p.im + (T)(s * y[2 * i + 1])};
  }
}

// training target t[v][k] = ((psi - psi0) / s_v) as (re, im)
template <typename T>
__global__ void k_pack_target(const Cx<T>* __restrict__ psi, const Cx<T>* __restrict__ psi0,
                              const float* __restrict__ scale, float* __restrict__ t, size_t n) {
  const int v = blockIdx.y;
  const float s = scale[v];
  const float inv = s > 0.f ? 1.f / s : 0.f;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const size_t i = (size_t)v * n + k;
    t[2 * i] = (float)(psi[i].re - psi0[i].re) * inv;
    t[2 * i + 1] = (float)(psi[i].im - psi0[i].im) * inv;
  }
}

// ------------------------------------------------------------------ launchers
namespace {
unsigned nn_grid(size_t count, size_t cap = 16384) {
  size_t g = (count + 255) / 256;
  if (g > cap) g = cap;
  return (unsigned)(g ? g : 1);
}
}  // namespace

hipError_t launch_conv_fwd(int ks, const float* X, int C, const unsigned short* Wb, int N, const float* bias, float* Y,
                           int B, int H, int W, bool relu, hipStream_t s) {
  const int P = B * H * W;
  if (P <= 0 || N <= 0) return hipSuccess;
  const dim3 grid((P + NN_T - 1) / NN_T, (N + NN_T - 1) / NN_T);
  const bool vec = C % 8 == 0 && ((uintptr_t)X % 16) == 0 && ((uintptr_t)Wb % 16) == 0;
  if (vec && ks == 3)
    hipLaunchKernelGGL(k_conv_fwd_v<3>, grid, dim3(256), 0, s, X, C, Wb, N, bias, Y, B, H, W, (int)relu);
  else if (vec && ks == 1)
    hipLaunchKernelGGL(k_conv_fwd_v<1>, grid, dim3(256), 0, s, X, C, Wb, N, bias, Y, B, H, W, (int)relu);
  else if (ks == 3)
    hipLaunchKernelGGL(k_conv_fwd<3>, grid, dim3(256), 0, s, X, C, Wb, N, bias, Y, B, H, W, (int)relu);
  else if (ks == 1)
    hipLaunchKernelGGL(k_conv_fwd<1>, grid, dim3(256), 0, s, X, C, Wb, N, bias, Y, B, H, W, (int)relu);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_conv_wgrad(int ks, const float* X, int C, const float* dY, int N, float* dW, int B, int H, int W,
                             hipStream_t s) {
  const int P = B * H * W, K = ks * ks * C;
  if (P <= 0) return hipSuccess;
  // pixel chunks: enough workgroups to fill the chip, chunks a multiple of the 32-pixel stage
  const int tiles = ((K + NN_T - 1) / NN_T) * ((N + NN_T - 1) / NN_T);
  int nz = std::max(1, std::min(1024, 2048 / std::max(1, tiles)));
  int pchunk = (P + nz - 1) / nz;
  pchunk = (pchunk + NN_K - 1) / NN_K * NN_K;
  nz = (P + pchunk - 1) / pchunk;
  const dim3 grid((K + NN_T - 1) / NN_T, (N + NN_T - 1) / NN_T, nz);
  const bool vec = C % 8 == 0 && N % 8 == 0 && ((uintptr_t)X % 16) == 0 && ((uintptr_t)dY % 16) == 0;
  if (vec && ks == 3)
    hipLaunchKernelGGL(k_conv_wgrad_v<3>, grid, dim3(256), 0, s, X, C, dY, N, dW, B, H, W, pchunk);
  else if (vec && ks == 1)
    hipLaunchKernelGGL(k_conv_wgrad_v<1>, grid, dim3(256), 0, s, X, C, dY, N, dW, B, H, W, pchunk);
  else if (ks == 3)
    hipLaunchKernelGGL(k_conv_wgrad<3>, grid, dim3(256), 0, s, X, C, dY, N, dW, B, H, W, pchunk);
  else if (ks == 1)
    hipLaunchKernelGGL(k_conv_wgrad<1>, grid, dim3(256), 0, s, X, C, dY, N, dW, B, H, W, pchunk);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_colsum(const float* dY, int P, int N, float* db, hipStream_t s) {
  if (P <= 0 || N <= 0) return hipSuccess;
  if (N <= 256) {
    const int pchunk = std::max(64, (P + 2047) / 2048);
    hipLaunchKernelGGL(k_colsum_flat, dim3((P + pchunk - 1) / pchunk), dim3(256), 0, s, dY, P, N, pchunk, db);
    return hipGetLastError();
  }
  const int bchunk = 1024;
  hipLaunchKernelGGL(k_colsum, dim3((N + 63) / 64, (P + bchunk - 1) / bchunk), dim3(64), 0, s, dY, P, N, bchunk, db);
  return hipGetLastError();
}

hipError_t launch_scale_copy(float* out, const float* z, size_t n, int stride, float scale, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_copy, dim3(nn_grid(n, 4096)), dim3(256), 0, s, out, z, n, stride, scale);
  return hipGetLastError();
}

hipError_t launch_relu_bwd(float* g, const float* y, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_relu_bwd, dim3(nn_grid(n)), dim3(256), 0, s, g, y, n);
  return hipGetLastError();
}

hipError_t launch_avgpool2(const float* x, float* y, int B, int h, int w, int C, hipStream_t s) {
  hipLaunchKernelGGL(k_avgpool2, dim3(nn_grid((size_t)B * h * w * C)), dim3(256), 0, s, x, y, B, h, w, C);
  return hipGetLastError();
}

hipError_t launch_avgpool2_bwd(const float* dy, const float* add, float* dx, int B, int h, int w, int C,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_avgpool2_bwd, dim3(nn_grid((size_t)B * 4 * h * w * C)), dim3(256), 0, s, dy, add, dx, B, h, w,
                     C);
  return hipGetLastError();
}

hipError_t launch_upcat(const float* lo, const float* skip, float* out, int B, int h, int w, int Cu, int Cs,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_upcat, dim3(nn_grid((size_t)B * 4 * h * w * (Cu + Cs))), dim3(256), 0, s, lo, skip, out, B, h,
                     w, Cu, Cs);
  return hipGetLastError();
}

hipError_t launch_upcat_bwd(const float* dcat, float* dlo, float* dskip, int B, int h, int w, int Cu, int Cs,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_upcat_bwd, dim3(nn_grid((size_t)B * h * w * (Cu + 4 * Cs))), dim3(256), 0, s, dcat, dlo, dskip,
                     B, h, w, Cu, Cs);
  return hipGetLastError();
}

hipError_t launch_mse(const float* out, const float* t, float* dout, size_t n, double* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_mse, dim3(nn_grid(n, 4096)), dim3(256), 0, s, out, t, dout, n, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* P, const float* G, float* M, float* V, size_t n, float lr, double b1, double b2,
                       double eps, int step, hipStream_t s) {
  const float c1 = (float)(1.0 - std::pow(b1, step)), c2 = (float)(1.0 - std::pow(b2, step));
  hipLaunchKernelGGL(k_adam, dim3(nn_grid(n)), dim3(256), 0, s, P, G, M, V, n, lr, (float)b1, (float)(1.0 - b1),
                     (float)b2, (float)(1.0 - b2), (float)eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_weights_bf16(const float* Wf, int ks, int Ci, int Co, unsigned short* Wb, unsigned short* WT,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_weights_bf16, dim3(nn_grid((size_t)ks * ks * Ci * Co)), dim3(256), 0, s, Wf, ks, Ci, Co, Wb,
                     WT);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pack_inputs(const double* chi, const Cx<T>* psi0, const double* norm2, float* out, int nvec,
                              size_t n, double c0w2, float k0h, float* scale, hipStream_t s) {
  if (nvec <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_pack_inputs<T>), dim3(nn_grid(n, 1024), nvec), dim3(256), 0, s, chi, psi0, norm2, out, n,
                     c0w2, k0h, scale);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_unpack_output(const Cx<T>* psi0, const float* y, const float* scale, Cx<T>* psi, int nvec, size_t n,
                                hipStream_t s) {
  if (nvec <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_unpack_output<T>), dim3(nn_grid(n, 1024), nvec), dim3(256), 0, s, psi0, y, scale, psi, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pack_target(const Cx<T>* psi, const Cx<T>* psi0, const float* scale, float* t, int nvec, size_t n,
                              hipStream_t s) {
  if (nvec <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_pack_target<T>), dim3(nn_grid(n, 1024), nvec), dim3(256), 0, s, psi, psi0, scale, t, n);
  return hipGetLastError();
}

template hipError_t launch_pack_target<float>(const Cx<float>*, const Cx<float>*, const float*, float*, int, size_t,
                                              hipStream_t);
template hipError_t launch_pack_target<double>(const Cx<double>*, const Cx<double>*, const float*, float*, int,
                                               size_t, hipStream_t);
template hipError_t launch_pack_inputs<float>(const double*, const Cx<float>*, const double*, float*, int, size_t,
                                              double, float, float*, hipStream_t);
template hipError_t launch_pack_inputs<double>(const double*, const Cx<double>*, const double*, float*, int, size_t,
                                               double, float, float*, hipStream_t);
template hipError_t launch_unpack_output<float>(const Cx<float>*, const float*, const float*, Cx<float>*, int, size_t,
                                                hipStream_t);
template hipError_t launch_unpack_output<double>(const Cx<double>*, const float*, const float*, Cx<double>*, int,
                                                 size_t, hipStream_t);

}  // namespace lsop
