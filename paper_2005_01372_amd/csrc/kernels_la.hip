// Dense linear algebra of the randomized preconditioner (Section 2.3):
// inner products W^H X over the n cells (split over n, FP64 accumulation),
// low-rank updates Y = X + U M, orthonormalisation of the range basis
// (Cholesky-QR run twice in the metric of the Gram matrix, with numerically
// dependent columns dropped), the r x r inverse Z = (I - W^H U)^{-1} of
// eq. (12) by Gauss-Jordan elimination with partial pivoting, Gaussian probes
// from Philox4x32-10, and small vector kernels.
#include "internal.hpp"

namespace lsop {

// ----------------------------------------------------------- vector kernels
template <typename T>
__global__ void k_norm2(const Cx<T>* __restrict__ x, double* __restrict__ out, const int* __restrict__ vidx,
                        size_t n) {
  const int slot = blockIdx.y;
  const int vi = vidx ? vidx[slot] : slot;
  const Cx<T>* xv = x + (size_t)vi * n;
  double s = 0.0;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const Cx<T> v = xv[k];
    s += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  __shared__ double red[16];
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  if (l == 0) red[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x / 64); ++i) t += red[i];
    atomicAdd(&out[slot], t);
  }
}

template <typename To, typename Ti>
__global__ void k_convert(const Cx<Ti>* __restrict__ x, Cx<To>* __restrict__ y, size_t count) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x)
    y[k] = ccast<To>(x[k]);
}

// y = a x + b y; with b = 0 the old y is not read (it may hold uninitialised values)
template <typename T>
__global__ void k_axpby(const Cx<T>* __restrict__ x, Cx<T>* __restrict__ y, T a, T b, const int* __restrict__ vidx,
                        size_t n) {
  const int slot = blockIdx.y;
  const size_t off = (size_t)(vidx ? vidx[slot] : slot) * n;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const Cx<T> xv = a != T(0) ? x[off + k] : czero<T>();
    const Cx<T> yv = b != T(0) ? y[off + k] : czero<T>();
    y[off + k] = Cx<T>{a * xv.re + b * yv.re, a * xv.im + b * yv.im};
  }
}

// p[k] = 0 for k < count (a fill kernel: usable inside captured graphs)
__global__ void k_zero_f64(double* __restrict__ p, size_t count) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x)
    p[k] = 0.0;
}

// tab[s].y[0 .. n) = 0 for the slots whose live[s] == 0 (frozen vectors of a grouped series)
template <typename T>
__global__ void k_mask_slots(const Slot<T>* __restrict__ tab, const int* __restrict__ live, size_t n) {
  const int sl = blockIdx.y;
  if (live[sl]) return;
  Cx<T>* y = tab[sl].y;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    y[k] = czero<T>();
}

// y[yidx[v]] += a * x[v] (x compact, y through the index list)
template <typename T>
__global__ void k_axpy_map(const Cx<T>* __restrict__ x, Cx<T>* __restrict__ y, const int* __restrict__ yidx, T a,
                           size_t n) {
  const int v = blockIdx.y;
  const Cx<T>* xv = x + (size_t)v * n;
  Cx<T>* yv = y + (size_t)(yidx ? yidx[v] : v) * n;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const Cx<T> xx = xv[k];
    const Cx<T> yy = yv[k];
    yv[k] = Cx<T>{yy.re + a * xx.re, yy.im + a * xx.im};
  }
}

template <typename T>
__global__ void k_accumulate(const Cx<T>* __restrict__ x, Cx<double>* __restrict__ y, double alpha,
                             const int* __restrict__ vidx, size_t n) {
  const int slot = blockIdx.y;
  const size_t off = (size_t)(vidx ? vidx[slot] : slot) * n;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    y[off + k] = y[off + k] + alpha * ccast<double>(x[off + k]);
}

template <typename T>
__global__ void k_real_to_complex(const double* __restrict__ in, Cx<T>* __restrict__ out, size_t count) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x)
    out[k] = Cx<T>{(T)in[k], T(0)};
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): 10 rounds of
// (hi0,lo0) = M0*c0, (hi1,lo1) = M1*c2, c <- (hi1^c1^k0, lo1, hi0^c3^k1, lo0),
// with the key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Probe k, pair t (elements 2t, 2t+1): counter (t lo, t hi, k, 0), key = seed;
// u1 = (x0 + 1/2) 2^-32, u2 = (x1 + 1/2) 2^-32, Box-Muller in FP64.
template <typename T>
__global__ void k_philox_normal(Cx<T>* __restrict__ out, size_t n, uint64_t seed, int k0) {
  const int k = k0 + blockIdx.y;
  const size_t npairs = (n + 1) / 2;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < npairs; t += (size_t)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)(t & 0xffffffffu), (uint32_t)(t >> 32), (uint32_t)k, 0u};
    philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    const double u1 = ((double)c[0] + 0.5) * 2.3283064365386962890625e-10;
    const double u2 = ((double)c[1] + 0.5) * 2.3283064365386962890625e-10;
    const double r = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    Cx<T>* o = out + (size_t)blockIdx.y * n;
    o[2 * t] = Cx<T>{(T)(r * cs), T(0)};
    if (2 * t + 1 < n) o[2 * t + 1] = Cx<T>{(T)(r * sn), T(0)};
  }
}

// ---------------------------------------------------------- C = A^H B (split over n)
// C[sg][k] = alpha * sum over the ksub partials of segment sg (part[sg * ksub + p][k]).
// C = alpha * (sum of the ksub partials) per segment; with C32 != NULL the FP64 sum is written rounded to FP32
// there instead.
__global__ void k_reduce_parts(const Cx<double>* __restrict__ part, int ksub, int nseg, size_t count,
                               Cx<double>* __restrict__ C, double alpha, Cx<float>* __restrict__ C32) {
  const size_t total = count * nseg;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t sg = idx / count, k = idx % count;
    const Cx<double>* p0 = part + sg * ksub * count + k;
    Cx<double> s = czero<double>();
    for (int p = 0; p < ksub; ++p) s = s + p0[(size_t)p * count];
    if (C32) C32[idx] = ccast<float>(alpha * s);
    else C[idx] = alpha * s;
  }
}

// ---------------------------------------------------------------- MFMA tiles
// v_mfma_*_16x16x4: A operand lane l = A[l % 16][l / 16], B operand lane l =
// B[l / 16][l % 16]; the 16 x 16 result row held in register r of lane l is
// 4 (l / 16) + r for f32 and 4 r + l / 16 for f64 (checked on gfx950), the
// column is l % 16.  A complex product is two real chains over interleaved
// (re, im) operands: with A'[.][2k + p] the p-th component of a_k,
//   conj(a) b:  re = sum_kk A'[kk] (br, bi)[kk],  im = sum_kk A'[kk] (bi, -br)[kk]
//   m a (no conj, m on the left):  re = (mr, -mi) . (ar, ai),  im = (mi, mr) . (ar, ai).
// The complex FP32 kernels below (segmented inner product, tile-form update, batched GEMM) instead take
// three real products per complex one (Gauss's 3M form): over complex k, t1 = sum ar br, t2 = sum ai bi and
// t3 = sum (ar - ai)(br + bi) give conj(a) b = (t1 + t2, t3 - t1 + t2); with t3 = sum (ar + ai)(br + bi),
// a b = (t1 - t2, t3 - t1 - t2).  Three quarters of the matrix-core work of the two chains.
typedef float lsop_f4 __attribute__((ext_vector_type(4)));
typedef double lsop_d4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  using acc = lsop_f4;
  __device__ __forceinline__ static acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <>
struct Mfma<double> {
  using acc = lsop_d4;
  __device__ __forceinline__ static acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int l, int r) { return 4 * r + (l >> 4); }
};

// C[a][b] partials = sum_k conj(A[a][k]) B[vb][k] over one k-chunk.  Tile
// 64 (a) x 64 (b) per workgroup of four waves (each 32 x 32 = 2 x 2 MFMA
// tiles; three chains of the 3M form in FP32, real and imaginary chains in FP64);
// operands staged in LDS 16 complex k at a time.
// The k range is cut into segments of `seg` elements (block-diagonal inner
// products: one result per segment), each into ksub chunks; z-block ks covers
// chunk ks % ksub of segment ks / ksub.
constexpr int GM_T = 64, GM_K = 16;

// Logical index of workgroup `id` of `total` such that consecutive logical
// indices run on the same XCD: workgroups are handed out round-robin over the
// 8 XCDs, each with its own L2, so XCD x takes the contiguous logical range
// [x total / 8, (x + 1) total / 8) (a bijection when total % 8 == 0; identity
// otherwise).  Workgroups that share operands (one segment's tiles) then
// share an L2.
// four reals as one vector (16 bytes for float; the FP64 instantiations never take the vector path)
template <typename T>
struct Vec4 {
  using type = float4;
};
template <>
struct Vec4<double> {
  struct type {
    double x, y, z, w;
  };
};

__device__ __forceinline__ unsigned xcd_block(unsigned id, unsigned total) {
  return (total % 8u) ? id : (id % 8u) * (total / 8u) + id / 8u;
}

// BT: the b extent of a workgroup's tile, 64 (four waves of 32 x 32 = 2 x 2 MFMA tiles) or 16 for at most 16
// vectors (four waves of 16 a x 16 b: a 64-wide b tile would leave three quarters of its MFMAs on zeros).
template <typename T, int BT>
__device__ __forceinline__ void ah_b_body(const Cx<T>* __restrict__ A, int na, const Cx<T>* __restrict__ B,
                                          const int* __restrict__ vidx, int nb, size_t n, size_t seg, size_t chunk,
                                          int ksub, Cx<double>* __restrict__ part, Cx<float>* __restrict__ out32) {
  using M = Mfma<T>;
  constexpr int NI = BT == GM_T ? 2 : 1, NJ = NI;
  // reals per LDS row: an even stride, so that (re, im) pairs are stored and read as one aligned pair (the 16
  // row offsets 34 c mod 64 banks are still distinct)
  constexpr int SROW = 2 * GM_K + 2;
  __shared__ __align__(16) T sa[GM_T * SROW];
  __shared__ __align__(16) T sb[BT * SROW];
  const unsigned lid = xcd_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                 gridDim.x * gridDim.y * gridDim.z);
  const int a0 = (int)(lid % gridDim.x) * GM_T, b0 = (int)((lid / gridDim.x) % gridDim.y) * BT;
  const int ks = (int)(lid / (gridDim.x * gridDim.y));
  const size_t seg_b = (size_t)(ks / ksub) * seg;
  const size_t seg_e = seg_b + seg < n ? seg_b + seg : n;
  const size_t k_begin = seg_b + (size_t)(ks % ksub) * chunk;
  const size_t k_end = k_begin + chunk < seg_e ? k_begin + chunk : seg_e;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wa = BT == GM_T ? (w >> 1) * 32 : w * 16, wb = BT == GM_T ? (w & 1) * 32 : 0;
  constexpr bool G3 = sizeof(T) == 4;  // 3M form (FP32)
  typename M::acc cre[NI][NJ], cim[NI][NJ], c3[G3 ? NI : 1][G3 ? NJ : 1];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      cre[i][j] = typename M::acc{0, 0, 0, 0};
      cim[i][j] = typename M::acc{0, 0, 0, 0};
      if constexpr (G3) c3[i][j] = typename M::acc{0, 0, 0, 0};
    }
  // loader: thread t -> row t / 4, complex k (t % 4) * 4 .. +4
  const int lr = threadIdx.x >> 2, lk = (threadIdx.x & 3) * 4;
  const Cx<T>* arow = (a0 + lr < na) ? A + (size_t)(a0 + lr) * n : nullptr;
  const int vb = b0 + lr;
  const Cx<T>* brow = (lr < BT && vb < nb) ? B + (size_t)(vidx ? vidx[vb] : vb) * n : nullptr;
  const int kk = l >> 4, c16 = l & 15;
  // the next stage's operands are loaded into registers while the current stage's MFMAs run; complex FP32
  // runs of 4 in range are loaded 16 bytes at a time (aligned when A and B are 16-byte aligned and n and
  // k_begin are even, since then row * n + k is even for every row and stage)
  Cx<T> va[4], vb2[4];
  const bool vec = sizeof(T) == 4 && ((n | k_begin) & 1) == 0 &&
                   ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0;
  auto load = [&](size_t kb) {
    const size_t k0 = kb + lk;
    if (vec && k0 + 4 <= k_end) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        using V = typename Vec4<T>::type;
        const V x = arow ? *reinterpret_cast<const V*>(arow + k0 + 2 * h) : V{0, 0, 0, 0};
        const V y = brow ? *reinterpret_cast<const V*>(brow + k0 + 2 * h) : V{0, 0, 0, 0};
        va[2 * h] = Cx<T>{x.x, x.y};
        va[2 * h + 1] = Cx<T>{x.z, x.w};
        vb2[2 * h] = Cx<T>{y.x, y.y};
        vb2[2 * h + 1] = Cx<T>{y.z, y.w};
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const size_t k = k0 + q;
        const bool kin = k < k_end;
        va[q] = (arow && kin) ? arow[k] : czero<T>();
        vb2[q] = (brow && kin) ? brow[k] : czero<T>();
      }
    }
  };
  load(k_begin);
  for (size_t kb = k_begin; kb < k_end; kb += GM_K) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *reinterpret_cast<Cx<T>*>(&sa[lr * SROW + 2 * (lk + q)]) = va[q];
      if (lr < BT) *reinterpret_cast<Cx<T>*>(&sb[lr * SROW + 2 * (lk + q)]) = vb2[q];
    }
    __syncthreads();
    if (kb + GM_K < k_end) load(kb + GM_K);
    if constexpr (G3) {
      // lane (c16, kk) takes complex k = 4 st + kk: cre, cim, c3 accumulate t1, t2, t3
#pragma unroll
      for (int st = 0; st < GM_K / 4; ++st) {
        const int col = 2 * (4 * st + kk);
        T ar[NI], ai[NI], as[NI], br[NJ], bi[NJ], bs[NJ];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          const Cx<T> v = *reinterpret_cast<const Cx<T>*>(&sa[(wa + i * 16 + c16) * SROW + col]);
          ar[i] = v.re;
          ai[i] = v.im;
          as[i] = v.re - v.im;
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const Cx<T> v = *reinterpret_cast<const Cx<T>*>(&sb[(wb + j * 16 + c16) * SROW + col]);
          br[j] = v.re;
          bi[j] = v.im;
          bs[j] = v.re + v.im;
        }
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            cre[i][j] = M::mma(ar[i], br[j], cre[i][j]);
            cim[i][j] = M::mma(ai[i], bi[j], cim[i][j]);
            c3[i][j] = M::mma(as[i], bs[j], c3[i][j]);
          }
      }
      __syncthreads();
      continue;
    }
#pragma unroll
    for (int st = 0; st < GM_K / 2; ++st) {
      const int col = 4 * st + kk;
      T av[NI], bre[NJ], bim[NJ];
#pragma unroll
      for (int i = 0; i < NI; ++i) av[i] = sa[(wa + i * 16 + c16) * SROW + col];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const Cx<T> v = *reinterpret_cast<const Cx<T>*>(&sb[(wb + j * 16 + c16) * SROW + (col & ~1)]);
        bre[j] = (kk & 1) ? v.im : v.re;
        bim[j] = (kk & 1) ? -v.re : v.im;
      }
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          cre[i][j] = M::mma(av[i], bre[j], cre[i][j]);
          cim[i][j] = M::mma(av[i], bim[j], cim[i][j]);
        }
    }
    __syncthreads();
  }
  if constexpr (G3) {
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const typename M::acc t1 = cre[i][j], t2 = cim[i][j];
        cre[i][j] = t1 + t2;
        cim[i][j] = c3[i][j] - t1 + t2;
      }
  }
  // one chunk per segment with out32: the partial is the product, written rounded to FP32
  Cx<double>* p = part + (size_t)ks * na * nb;
  Cx<float>* p32 = out32 ? out32 + (size_t)ks * na * nb : nullptr;
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = a0 + wa + i * 16 + M::row(l, r);
        const int b = b0 + wb + j * 16 + c16;
        if (a < na && b < nb) {
          if (out32) p32[(size_t)a * nb + b] = Cx<float>{(float)cre[i][j][r], (float)cim[i][j][r]};
          else p[(size_t)a * nb + b] = Cx<double>{(double)cre[i][j][r], (double)cim[i][j][r]};
        }
      }
}

// complex FP32 at 5 waves per SIMD (96 registers, no spills; 4 without the hint)
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 1))) void
k_gemm_ah_b_mfma(const Cx<T>* __restrict__ A, int na, const Cx<T>* __restrict__ B, const int* __restrict__ vidx, int nb,
                 size_t n, size_t seg, size_t chunk, int ksub, Cx<double>* __restrict__ part,
                 Cx<float>* __restrict__ out32) {
  ah_b_body<T, GM_T>(A, na, B, vidx, nb, n, seg, chunk, ksub, part, out32);
}

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_ah_b_narrow(const Cx<T>* __restrict__ A, int na,
                                                          const Cx<T>* __restrict__ B, const int* __restrict__ vidx,
                                                          int nb, size_t n, size_t seg, size_t chunk, int ksub,
                                                          Cx<double>* __restrict__ part,
                                                          Cx<float>* __restrict__ out32) {
  ah_b_body<T, 16>(A, na, B, vidx, nb, n, seg, chunk, ksub, part, out32);
}

// Y[vy(b)][k] = X1 + beta X2 + sum_a A[a][k] M[a][b] as out[b][k] = M^T A
// (segmented form: M for element k is M + (k / seg) * mstride; M in MT, FP64 or T, rounded to T in LDS):
// each wave owns 16 consecutive k (coalesced B-operand loads and stores) and
// up to NBT * 16 b (MFMA row tiles, real and imaginary chains); M is staged in
// LDS GA rows (a) at a time; the A elements and the M rows of the next
// block are loaded into registers while the current block's MFMAs run (a
// whole block in flight per lane covers the memory latency; short blocks keep
// the register count, and so the occupancy, up).  GA rows per block; WPE > 0
// asks the compiler for that many waves per SIMD (complex float, 64-wide b
// passes: 4-row blocks at 6 waves run 12% faster than 8-row blocks at the
// default 4 waves, bit-identical; measured over na = 64-256, nb = 40-256;
// complex double: 4-row blocks at 3 waves remove the 8-row form's spills).
template <typename T, typename MT, int NBT, int GA, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1))) void k_gemm_update_mfma(
    const Cx<T>* A, int na,
                                                          const Cx<MT>* __restrict__ Mm, int nb,
                                                          const Cx<T>* X1, const Cx<T>* X2, T beta, Cx<T>* Y,
                                                          const int* __restrict__ vidx, size_t n, size_t seg,
                                                          size_t mstride) {
  using MF = Mfma<T>;
  constexpr int BW = NBT * 16;
  __shared__ Cx<T> sm[GA * BW];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const size_t bx = xcd_block(blockIdx.x, gridDim.x);
  const size_t k0 = (bx * 4 + w) * 16;
  // segmented form: the workgroup's 64 elements lie in one segment (seg % 64 == 0)
  Mm += (bx * 64 / seg) * mstride;
  const int kk = l >> 4, c16 = l & 15, pp = kk & 1;
  const size_t kcol = k0 + c16;
  const bool kin = kcol < n;
  for (int b0 = 0; b0 < nb; b0 += BW) {
    typename MF::acc cre[NBT], cim[NBT];
#pragma unroll
    for (int j = 0; j < NBT; ++j) {
      cre[j] = typename MF::acc{0, 0, 0, 0};
      cim[j] = typename MF::acc{0, 0, 0, 0};
    }
    // lane's A elements of one block: a = a0 + 2 st + kk / 2, st < GA / 2; the thread's share of the
    // M block (PER elements, idx = threadIdx.x + 256 q); both loaded one block ahead of their use
    constexpr int PER = (GA * BW + 255) / 256;
    const int ab = kk >> 1;
    Cx<T> av[GA / 2];
    Cx<MT> mv[PER];
#pragma unroll
    for (int st = 0; st < GA / 2; ++st) {
      const int a = ab + 2 * st;
      av[st] = (kin && a < na) ? A[(size_t)a * n + kcol] : czero<T>();
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = threadIdx.x + 256 * q, a = idx / BW, b = b0 + idx % BW;
      mv[q] = (idx < GA * BW && a < na && b < nb) ? Mm[(size_t)a * nb + b] : czero<MT>();
    }
    for (int a0 = 0; a0 < na; a0 += GA) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < PER; ++q)
        if (threadIdx.x + 256 * q < GA * BW) sm[threadIdx.x + 256 * q] = ccast<T>(mv[q]);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int idx = threadIdx.x + 256 * q, a = a0 + GA + idx / BW, b = b0 + idx % BW;
        mv[q] = (idx < GA * BW && a < na && b < nb) ? Mm[(size_t)a * nb + b] : czero<MT>();
      }
      Cx<T> cur[GA / 2];
#pragma unroll
      for (int st = 0; st < GA / 2; ++st) cur[st] = av[st];
#pragma unroll
      for (int st = 0; st < GA / 2; ++st) {
        const int a = a0 + GA + ab + 2 * st;
        av[st] = (kin && a < na) ? A[(size_t)a * n + kcol] : czero<T>();
      }
#pragma unroll
      for (int st = 0; st < GA / 2; ++st) {
        const T bop = pp ? cur[st].im : cur[st].re;
        const int al = 2 * st + (kk >> 1);
#pragma unroll
        for (int j = 0; j < NBT; ++j) {
          const Cx<T> m = sm[al * BW + j * 16 + c16];
          const T ore = pp ? -m.im : m.re;
          const T oim = pp ? m.re : m.im;
          cre[j] = MF::mma(ore, bop, cre[j]);
          cim[j] = MF::mma(oim, bop, cim[j]);
        }
      }
    }
    if (kin) {
#pragma unroll
      for (int j = 0; j < NBT; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int b = b0 + j * 16 + MF::row(l, r);
          if (b < nb) {
            const size_t off = (size_t)(vidx ? vidx[b] : b) * n + kcol;
            Cx<T> out{cre[j][r], cim[j][r]};
            if (X1) out = out + X1[off];
            if (X2) out = out + beta * X2[off];
            Y[off] = out;
          }
        }
    }
  }
}

// GEMM-tile form of the same update for complex float and nb > 32: a workgroup owns a 64 (b) x 64 (k) tile of Y
// (four waves of 32 x 32 = 2 x 2 MFMA tiles, three chains of the 3M form); M (rounded to FP32) and A are both
// staged in LDS 16 complex a at a time, the next stage loaded into registers while the current stage's MFMAs
// run, so a barrier pair covers 48 MFMAs per wave.  The tiles of one 64-element k range follow each other on one
// XCD, so A's re-reads by its b tiles are L2 hits.  LDS rows of 80 complex put the a rows that one MFMA operand
// spans 32 banks apart in turn.  Measured at n = 1M (standalone, two-chain form, against the per-wave form
// above): na = 256, nb = 128-256 with FP32 M at 6 waves per SIMD 108 -> 118 TFLOP/s; na = 64-192, nb = 64 with
// FP64 M (no occupancy hint; 6 waves was slower there) 76 -> 86 and 97 -> 110 TFLOP/s.  The 3M form needs 16
// more registers (10 spilled at 6 waves); both instantiations run at 5 waves per SIMD.
constexpr int UPD_T = 64, UPD_K = 16, UPD_ROW = UPD_T + 16;
template <typename MT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void
k_gemm_update_tile(const Cx<float>* A, int na, const Cx<MT>* __restrict__ Mm, int nb,
                   const Cx<float>* X1, const Cx<float>* X2, float beta, Cx<float>* Y,
                   const int* __restrict__ vidx, size_t n, size_t seg, size_t mstride) {
  using MF = Mfma<float>;
  __shared__ __align__(16) Cx<float> sm[UPD_K * UPD_ROW];
  __shared__ __align__(16) Cx<float> sx[UPD_K * UPD_ROW];
  const int nbt = (nb + UPD_T - 1) / UPD_T;
  const size_t lid = xcd_block(blockIdx.x, gridDim.x);
  const size_t k0 = (lid / nbt) * UPD_T;
  const int b0 = (int)(lid % nbt) * UPD_T;
  Mm += (k0 / seg) * mstride;  // the tile's 64 elements lie in one segment (seg % 64 == 0)
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wb = (w >> 1) * 32, wk = (w & 1) * 32;
  // loader: thread t -> stage row t / 16, columns lj, lj + 1 and 32 + lj, 33 + lj (lj = 2 (t % 16)), each pair
  // stored to LDS as 16 bytes: the 16 lanes of a store pass then cover the 64 banks once (with four consecutive
  // columns per thread, lanes 8 apart met on the same banks), and each global load stays 256 contiguous bytes
  const int la = threadIdx.x >> 4, lj = (threadIdx.x & 15) * 2;
  auto lcol = [&](int q) { return lj + (q & 1) + 32 * (q >> 1); };
  // operand lanes: kk = l / 16 is the MFMA's k index, complex a = 4 st + kk.  Gauss's 3M form: t1 = sum mr xr,
  // t2 = sum mi xi, t3 = sum (mr + mi)(xr + xi) in c1, c2, c3; m x = (t1 - t2, t3 - t1 - t2).
  const int kk = l >> 4, c16 = l & 15;
  typename MF::acc c1[2][2], c2[2][2], c3[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      c1[i][j] = typename MF::acc{0, 0, 0, 0};
      c2[i][j] = typename MF::acc{0, 0, 0, 0};
      c3[i][j] = typename MF::acc{0, 0, 0, 0};
    }
  Cx<MT> vm[4];
  Cx<float> vx[4];
  const bool vec = (n & 1) == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0 && k0 + UPD_T <= n;
  auto load = [&](int a0) {
    const int a = a0 + la;
    const bool ain = a < na;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = b0 + lcol(q);
      vm[q] = (ain && b < nb) ? Mm[(size_t)a * nb + b] : czero<MT>();
    }
    if (vec) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float4 x = ain ? *reinterpret_cast<const float4*>(A + (size_t)a * n + k0 + lj + 32 * h)
                             : float4{0.f, 0.f, 0.f, 0.f};
        vx[2 * h] = Cx<float>{x.x, x.y};
        vx[2 * h + 1] = Cx<float>{x.z, x.w};
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const size_t k = k0 + lcol(q);
        vx[q] = (ain && k < n) ? A[(size_t)a * n + k] : czero<float>();
      }
    }
  };
  load(0);
  for (int a0 = 0; a0 < na; a0 += UPD_K) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const Cx<float> m0 = ccast<float>(vm[2 * h]), m1 = ccast<float>(vm[2 * h + 1]);
      *reinterpret_cast<float4*>(&sm[la * UPD_ROW + lj + 32 * h]) = float4{m0.re, m0.im, m1.re, m1.im};
      *reinterpret_cast<float4*>(&sx[la * UPD_ROW + lj + 32 * h]) =
          float4{vx[2 * h].re, vx[2 * h].im, vx[2 * h + 1].re, vx[2 * h + 1].im};
    }
    __syncthreads();
    if (a0 + UPD_K < na) load(a0 + UPD_K);
#pragma unroll
    for (int st = 0; st < UPD_K / 4; ++st) {
      const int ar = 4 * st + kk;
      float mr[2], mi[2], ms[2], xr[2], xi[2], xs[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const Cx<float> m = sm[ar * UPD_ROW + wb + i * 16 + c16];
        mr[i] = m.re;
        mi[i] = m.im;
        ms[i] = m.re + m.im;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const Cx<float> x = sx[ar * UPD_ROW + wk + j * 16 + c16];
        xr[j] = x.re;
        xi[j] = x.im;
        xs[j] = x.re + x.im;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          c1[i][j] = MF::mma(mr[i], xr[j], c1[i][j]);
          c2[i][j] = MF::mma(mi[i], xi[j], c2[i][j]);
          c3[i][j] = MF::mma(ms[i], xs[j], c3[i][j]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int b = b0 + wb + i * 16 + MF::row(l, r);
        const size_t k = k0 + wk + j * 16 + c16;
        if (b < nb && k < n) {
          const size_t off = (size_t)(vidx ? vidx[b] : b) * n + k;
          const float t1 = c1[i][j][r], t2 = c2[i][j][r];
          Cx<float> out{t1 - t2, c3[i][j][r] - t1 - t2};
          if (X1) out = out + X1[off];
          if (X2) out = out + beta * X2[off];
          Y[off] = out;
        }
      }
}

// ------------------------------------------------------- small FP64 kernels
// Orthonormalising coefficients X (na x na, na <= 64) for Q = Y X from the
// Gram matrix G = Y^H Y: X = R^{-1} with G = R^H R (Cholesky), so that
// X^H G X = I.  A column whose Schur-complement diagonal (its G-norm^2 after
// projection on the kept earlier columns) is <= drop_tol * R_kk is dropped: its
// row of R and its column of X are zero and it takes no part in later
// eliminations; R_kk is gnorm[b][k] (the squared norm of column k before an
// earlier projection, na per batch entry) or G's own diagonal.  One workgroup
// of four waves per batch entry b (G_b, X_b at b * na * na, kept[b]).  The right-looking factorisation is run
// as row operations on [G | I] in LDS: step k scales row k by 1 / sqrt(d_k)
// (wave 0), then every later row i subtracts conj(R_ki) times it (rows split
// over the waves, lane = column); the upper triangle of the left block becomes
// R and the right block R^{-H} = X^H.  Two barriers per column.
constexpr int SMALL_NA = 64;

// out[sg * na + c] = sum over the segment's elements k of |Y[c][k]|^2, in FP64 (the reference norms of the
// drop test above): one workgroup per (column c, segment sg), workgroup id sg * na + c; a fixed summation order.
template <typename T>
__global__ __launch_bounds__(256) void k_seg_colnorm2(const Cx<T>* __restrict__ Y, int na, size_t n, size_t seg,
                                                       double* __restrict__ out) {
  const int c = (int)(blockIdx.x % (unsigned)na);
  const size_t sg = blockIdx.x / (unsigned)na;
  const size_t b = sg * seg, e = b + seg < n ? b + seg : n;
  const Cx<T>* y = Y + (size_t)c * n;
  double acc = 0.0;
  for (size_t k = b + threadIdx.x; k < e; k += blockDim.x) {
    const Cx<T> v = y[k];
    acc += (double)v.re * v.re + (double)v.im * v.im;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_gram_orth_lds(const Cx<double>* __restrict__ Gg, Cx<double>* __restrict__ Xg,
                                                        int na, double drop_tol, int* kept,
                                                        const double* __restrict__ gnorm) {
  constexpr int ES = SMALL_NA + 1;  // row stride of E (odd: the transposed read at the end is conflict-free)
  __shared__ Cx<double> S[SMALL_NA * SMALL_NA];  // G, reduced in place (upper triangle: R)
  __shared__ Cx<double> E[SMALL_NA * ES];        // I, taken to R^{-H} by the same row operations
  __shared__ double g0[SMALL_NA];                // reference diagonal of the drop test
  const size_t off = (size_t)blockIdx.x * na * na;
  const int t = threadIdx.x, j = t & 63, wv = t >> 6;
  for (int idx = t; idx < na * na; idx += blockDim.x) {
    const int i = idx / na, c = idx - i * na;
    S[i * SMALL_NA + c] = Gg[off + idx];
    E[i * ES + c] = Cx<double>{i == c ? 1.0 : 0.0, 0.0};
  }
  if (t < na) g0[t] = gnorm ? gnorm[(size_t)blockIdx.x * na + t] : Gg[off + (size_t)t * na + t].re;
  __syncthreads();
  int nkept = 0;
  for (int k = 0; k < na; ++k) {
    // pivot: d = remaining G-norm^2 of column k (every thread takes the same decision)
    const double d = S[k * SMALL_NA + k].re, g = g0[k];
    const bool keep = g > 1e-300 && d > drop_tol * g;
    nkept += keep ? 1 : 0;
    if (wv == 0 && j < na) {
      const double sc = keep ? 1.0 / sqrt(d) : 0.0;
      if (j > k) S[k * SMALL_NA + j] = sc * S[k * SMALL_NA + j];
      else E[k * ES + j] = sc * E[k * ES + j];
    }
    __syncthreads();
    if (keep && j < na) {
      // lane j's entry of row k: R_kj in the left block (j > k), E_kj in the right one (j <= k)
      const Cx<double> rk = j > k ? S[k * SMALL_NA + j] : E[k * ES + j];
      for (int i = k + 1 + wv; i < na; i += 4) {
        const Cx<double> c = S[k * SMALL_NA + i];
        const Cx<double> cc{c.re, -c.im};
        if (j >= i) S[i * SMALL_NA + j] = S[i * SMALL_NA + j] - cc * rk;
        else if (j <= k) E[i * ES + j] = E[i * ES + j] - cc * rk;
      }
    }
    __syncthreads();
  }
  for (int idx = t; idx < na * na; idx += blockDim.x) {
    const int i = idx / na, c = idx - i * na;
    const Cx<double> e = E[c * ES + i];
    Xg[off + idx] = Cx<double>{e.re, -e.im};
  }
  if (t == 0) kept[blockIdx.x] = nkept;
}

// max over the workgroup of (value, index), lowest index on ties; red / redi
// hold one entry per wavefront; the result is returned to every thread.
__device__ __forceinline__ void block_argmax(double v, int i, double* red, int* redi, double* vo, int* io) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o);
    const int oi = __shfl_xor(i, o);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
  const int nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = v;
    redi[threadIdx.x >> 6] = i;
  }
  __syncthreads();
  v = red[0];
  i = redi[0];
  for (int q = 1; q < nw; ++q)
    if (red[q] > v || (red[q] == v && redi[q] < i)) {
      v = red[q];
      i = redi[q];
    }
  *vo = v;
  *io = i;
  __syncthreads();
}

// Inverse by in-place Gauss-Jordan with partial pivoting of B = I - M (plain =
// 0, eq. 12) or B = M (plain = 1), held in work (row stride wld >= na).  Step k
// swaps the pivot row into place, scales it by 1 / pivot with the pivot slot
// set to 1 / pivot, and eliminates column k from every other row with the
// slot set to -(its entry) / pivot: column k of the array then holds column k
// of the inverse of the row-permuted matrix.  The row swaps are undone at the
// end as column swaps in reverse order (inv(P B) P = inv(B)).  M has leading
// dimension ldm, Z ldz (Z may alias M).  *singular is set to 1 on a vanishing
// pivot (never cleared here, so one flag can collect several calls).  fcol:
// na entries, perm: 2 na entries of shared memory.  T = double (pivot
// threshold 1e-14 of the largest entry) or float (1e-6).
template <typename T>
__device__ __forceinline__ void lu_inverse_body(const Cx<T>* M, size_t ldm, Cx<T>* Z, size_t ldz, Cx<T>* work,
                                                int wld, int na, int plain, int* singular, Cx<T>* fcol, int* perm,
                                                double* red, int* redi) {
  const double tiny = sizeof(T) == sizeof(double) ? 1e-14 : 1e-6;
  const int t = threadIdx.x, nt = blockDim.x;
  double amax = 0.0;
  for (int idx = t; idx < na * na; idx += nt) {
    const int i = idx / na, j = idx - i * na;
    const Cx<T> m = M[(size_t)i * ldm + j];
    const Cx<T> v = plain ? m : Cx<T>{(i == j ? T(1) : T(0)) - m.re, -m.im};
    work[(size_t)i * wld + j] = v;
    amax = fmax(amax, sqrt((double)norm2(v)));
  }
  double scale;
  int dummy;
  block_argmax(amax, 0, red, redi, &scale, &dummy);
  // elimination layout: thread t owns column uj = t % na of rows ui0, ui0 + urs, ... (no division in the loop);
  // urs = 0 (na > nt) falls back to a loop over columns
  const int urs = nt / na, uj = t % na, ui0 = t / na;
  for (int k = 0; k < na; ++k) {
    double bv = -1.0;
    int bi = k;
    for (int i = k + t; i < na; i += nt) {
      const double v = (double)norm2(work[(size_t)i * wld + k]);
      if (v > bv) {
        bv = v;
        bi = i;
      }
    }
    double piv2;
    int p;
    block_argmax(bv, bi, red, redi, &piv2, &p);
    if (!(sqrt(piv2) > tiny * scale)) {
      if (t == 0) *singular = 1;
      return;  // uniform across the workgroup
    }
    if (t == 0) perm[k] = p;
    if (p != k) {
      for (int j = t; j < na; j += nt) {
        const Cx<T> a = work[(size_t)k * wld + j];
        work[(size_t)k * wld + j] = work[(size_t)p * wld + j];
        work[(size_t)p * wld + j] = a;
      }
    }
    __syncthreads();
    const Cx<T> pv = work[(size_t)k * wld + k];
    const T d = T(1) / norm2(pv);
    const Cx<T> inv = Cx<T>{pv.re * d, -pv.im * d};
    __syncthreads();
    for (int j = t; j < na; j += nt)
      work[(size_t)k * wld + j] = (j == k ? Cx<T>{T(1), T(0)} : work[(size_t)k * wld + j]) * inv;
    for (int i = t; i < na; i += nt) fcol[i] = work[(size_t)i * wld + k];
    __syncthreads();
    if (urs > 0) {
      if (ui0 < urs) {
        const Cx<T> pr = work[(size_t)k * wld + uj];
        for (int i = ui0; i < na; i += urs)
          if (i != k)
            work[(size_t)i * wld + uj] = (uj == k ? czero<T>() : work[(size_t)i * wld + uj]) - fcol[i] * pr;
      }
    } else {
      for (int j = t; j < na; j += nt) {
        const Cx<T> pr = work[(size_t)k * wld + j];
        for (int i = 0; i < na; ++i)
          if (i != k) work[(size_t)i * wld + j] = (j == k ? czero<T>() : work[(size_t)i * wld + j]) - fcol[i] * pr;
      }
    }
    __syncthreads();
  }
  // column of the array that lands at column j of the inverse: the row swaps replayed backwards as column swaps
  int* pos = perm + na;
  if (t == 0) {
    for (int j = 0; j < na; ++j) pos[j] = j;
    for (int k = na - 1; k >= 0; --k) {
      const int q = perm[k], a = pos[k];
      pos[k] = pos[q];
      pos[q] = a;
    }
  }
  __syncthreads();
  for (int idx = t; idx < na * na; idx += nt) {
    const int i = idx / na, j = idx - i * na;
    Z[(size_t)i * ldz + j] = work[(size_t)i * wld + pos[j]];
  }
}

// Batch entry b = blockIdx.x: M + b * sm, Z + b * sz, singular[b].  The LDS
// work rows have an odd stride (conflict-free column reads).
constexpr int LU_WLD = SMALL_NA + 1;

template <typename T>
__global__ __launch_bounds__(256) void k_lu_inverse_lds(const Cx<T>* __restrict__ M, size_t ldm, size_t sm, Cx<T>* Z,
                                                         size_t ldz, size_t sz, int na, int plain, int* singular) {
  __shared__ Cx<T> work[SMALL_NA * LU_WLD];
  __shared__ Cx<T> fcol[SMALL_NA];
  __shared__ int perm[2 * SMALL_NA];
  __shared__ double red[4];
  __shared__ int redi[4];
  const size_t b = blockIdx.x;
  lu_inverse_body<T>(M + b * sm, ldm, Z + b * sz, ldz, work, LU_WLD, na, plain, singular + b, fcol, perm, red, redi);
}

// larger na: the work array in global memory (2 na^2 entries per batch entry, row stride 2 na); fcol and the
// permutation in dynamic shared memory (na complex + 2 na ints)
__global__ __launch_bounds__(256) void k_lu_inverse_i_minus(const Cx<double>* __restrict__ M, size_t ldm, size_t sm,
                                                             Cx<double>* Z, size_t ldz, size_t sz,
                                                             Cx<double>* __restrict__ work, int na, int plain,
                                                             int* singular) {
  extern __shared__ unsigned char smem_raw[];
  Cx<double>* fcol = reinterpret_cast<Cx<double>*>(smem_raw);   // [na]
  int* perm = reinterpret_cast<int*>(fcol + na);                 // [2 na]
  __shared__ double red[4];
  __shared__ int redi[4];
  const size_t b = blockIdx.x;
  lu_inverse_body<double>(M + b * sm, ldm, Z + b * sz, ldz, work + b * 2 * (size_t)na * na, 2 * na, na, plain,
                          singular + b, fcol, perm, red, redi);
}

// C_b = alpha * A_b (na x na) B_b (na x nb); batch entry b = blockIdx.y.
__global__ void k_small_gemm(const Cx<double>* __restrict__ A, const Cx<double>* __restrict__ B,
                             Cx<double>* __restrict__ C, int na, int nb, double alpha) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= na * nb) return;
  const size_t b = blockIdx.y;
  A += b * na * na;
  B += b * na * nb;
  C += b * na * nb;
  const int i = idx / nb, j = idx % nb;
  Cx<double> s = czero<double>();
  for (int l = 0; l < na; ++l) s = s + A[(size_t)i * na + l] * B[(size_t)l * nb + j];
  C[idx] = alpha * s;
}

// ------------------------------------------------- hierarchical (HODLR) kernels
// Dense diagonal leaf blocks of A = I - G0 V (eq. 5) for leaves of w grid
// columns (nl = w nz cells, column-wise order): out[b][a][c] =
// delta_ac - K(|ia - ic|, |ja - jc|) chi[c] for leaf leaf0 + b.
template <typename To>
__global__ void k_leaf_form(const Cx<double>* __restrict__ ktab, const double* __restrict__ chi,
                            Cx<To>* __restrict__ out, int nz, int nl, int leaf0, int nleaf) {
  const size_t per = (size_t)nl * nl, total = per * nleaf;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx / per);
    const size_t rem = idx % per;
    const int a = (int)(rem / nl), c = (int)(rem % nl);
    const int ia = a / nz, ja = a % nz, ic = c / nz, jc = c % nz;
    const int di = ia > ic ? ia - ic : ic - ia, dj = ja > jc ? ja - jc : jc - ja;
    const double x = chi[(size_t)(leaf0 + b) * nl + c];
    const Cx<double> k = ktab[(size_t)di * nz + dj];
    out[idx] = Cx<To>{(To)((a == c ? 1.0 : 0.0) - x * k.re), (To)(-x * k.im)};
  }
}

// out[b][j][i] = in[b][i][j] (Ti -> T), 32 x 32 tiles through LDS.
template <typename T, typename Ti = double>
__global__ __launch_bounds__(256) void k_transpose_convert(const Cx<Ti>* __restrict__ in, Cx<T>* __restrict__ out,
                                                            int m) {
  __shared__ Cx<Ti> tile[32][33];
  const size_t b = blockIdx.z;
  const Cx<Ti>* src = in + b * m * m;
  Cx<T>* dst = out + b * m * m;
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  for (int r = ty; r < 32; r += 8)
    if (i0 + r < m && j0 + tx < m) tile[r][tx] = src[(size_t)(i0 + r) * m + j0 + tx];
  __syncthreads();
  for (int r = ty; r < 32; r += 8)
    if (j0 + r < m && i0 + tx < m) dst[(size_t)(j0 + r) * m + i0 + tx] = ccast<T>(tile[tx][r]);
}

// out_b[i][j] = delta_ij for an r x r block (leading dimension ld, batch stride st)
__global__ void k_set_identity(Cx<double>* __restrict__ out, size_t ld, size_t st, int r, int batch) {
  const size_t per = (size_t)r * r, total = per * batch;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t b = idx / per;
    const int i = (int)(idx % per) / r, j = (int)(idx % per) % r;
    out[b * st + (size_t)i * ld + j] = Cx<double>{i == j ? 1.0 : 0.0, 0.0};
  }
}

// dev[b] = max_ij |P_b[i][j] - delta_ij| (one workgroup per batch entry)
__global__ __launch_bounds__(256) void k_identity_deviation(const Cx<double>* __restrict__ P, size_t ld, size_t st,
                                                             int r, double* __restrict__ dev) {
  const Cx<double>* pb = P + (size_t)blockIdx.x * st;
  double m = 0.0;
  for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {
    const int i = idx / r, j = idx % r;
    const Cx<double> v = pb[(size_t)i * ld + j];
    const double re = v.re - (i == j ? 1.0 : 0.0);
    m = fmax(m, sqrt(re * re + v.im * v.im));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) dev[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Batched complex GEMM on MFMA: C_b = alpha A_b B_b + beta C_b, row-major,
// A_b: M x K, B_b: K x N, C_b: M x N.  Row m of A is found at
// (mapa ? mapa[m] : m) * lda + b * sA, row m of C likewise through mapc (the
// maps address vectors of a batch through an index list).  Tile 64 x 64 per workgroup of four waves
// (2 x 2 MFMA tiles each, real and imaginary chains over interleaved (re, im)
// operands: re = sum (ar br - ai bi), im = sum (ar bi + ai br)).  Complex FP32 takes Gauss's 3M form
// instead: t1 = sum ar br, t2 = sum ai bi, t3 = sum (ar + ai)(br + bi), a b = (t1 - t2, t3 - t1 - t2).
template <typename T>
__global__ __launch_bounds__(256) void k_bgemm_mfma(const Cx<T>* A, size_t lda, size_t sA, const Cx<T>* B,
                                                    size_t ldb, size_t sB, Cx<T>* C, size_t ldc, size_t sC,
                                                    const int* __restrict__ mapa, const int* __restrict__ mapc, int M,
                                                    int N, int K, T alpha, T beta) {
  using MF = Mfma<T>;
  constexpr int SROW = 2 * GM_K + 2;  // even: (re, im) pairs stored and read as one aligned pair
  __shared__ __align__(16) T sa[GM_T * SROW];
  __shared__ __align__(16) T sb[GM_T * SROW];
  // all tiles of one batch entry (which share its A rows and B columns) at consecutive logical indices on
  // one XCD, so their re-reads of the operands are L2 hits
  const unsigned lid = xcd_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                 gridDim.x * gridDim.y * gridDim.z);
  const size_t bt = lid / (gridDim.x * gridDim.y);
  const int n0 = (int)(lid % gridDim.x) * GM_T, m0 = (int)((lid / gridDim.x) % gridDim.y) * GM_T;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  constexpr bool G3 = sizeof(T) == 4;  // 3M form (FP32)
  typename MF::acc cre[2][2], cim[2][2], c3[G3 ? 2 : 1][G3 ? 2 : 1];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cre[i][j] = typename MF::acc{0, 0, 0, 0};
      cim[i][j] = typename MF::acc{0, 0, 0, 0};
      if constexpr (G3) c3[i][j] = typename MF::acc{0, 0, 0, 0};
    }
  // A loader: thread t -> row t / 4, k (t % 4) * 4 .. +4 ; B loader: k t / 16 and four n, bn + BQ q (q < 4).
  // Complex FP32 takes four consecutive n (bn = 4 (t % 16), BQ = 1: two 16-byte loads); complex FP64, which
  // loads element-wise, takes bn = t % 16 and BQ = 16, so that its transposed LDS stores of a pass fall on
  // distinct banks (consecutive n put lanes 8 apart on the same banks; 3-4% faster).  For FP32 the 16-byte
  // loads weigh more than the conflicts: the element-wise form was 12% slower.
  constexpr int BQ = sizeof(T) == 4 ? 1 : 16;
  const int ar = threadIdx.x >> 2, ak = (threadIdx.x & 3) * 4;
  const int bk = threadIdx.x >> 4, bn = sizeof(T) == 4 ? (threadIdx.x & 15) * 4 : threadIdx.x & 15;
  const Cx<T>* arow = nullptr;
  if (m0 + ar < M) arow = A + bt * sA + (size_t)(mapa ? mapa[m0 + ar] : m0 + ar) * lda;
  const Cx<T>* bbase = B + bt * sB;
  const int kk = l >> 4, c16 = l & 15;
  // the next stage's operands are loaded into registers while the current stage's MFMAs run; complex FP32
  // runs of 4 (k of an A row, n of a B row) are loaded 16 bytes at a time when the entry's base is 16-byte
  // aligned and its row stride even (every run then starts at an even element)
  Cx<T> va[4], vb[4];
  using V = typename Vec4<T>::type;
  const bool veca = sizeof(T) == 4 && (lda & 1) == 0 && (reinterpret_cast<uintptr_t>(A + bt * sA) & 15) == 0;
  const bool vecb = sizeof(T) == 4 && (ldb & 1) == 0 && (reinterpret_cast<uintptr_t>(bbase) & 15) == 0;
  auto load = [&](int kb) {
    const int k0 = kb + ak, kb2 = kb + bk, nn0 = n0 + bn;
    if (veca && k0 + 4 <= K) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const V x = arow ? *reinterpret_cast<const V*>(arow + k0 + 2 * h) : V{0, 0, 0, 0};
        va[2 * h] = Cx<T>{x.x, x.y};
        va[2 * h + 1] = Cx<T>{x.z, x.w};
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) va[q] = (arow && k0 + q < K) ? arow[k0 + q] : czero<T>();
    }
    if (vecb && kb2 < K && nn0 + 4 <= N) {
      const Cx<T>* bp = bbase + (size_t)kb2 * ldb + nn0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const V y = *reinterpret_cast<const V*>(bp + 2 * h);
        vb[2 * h] = Cx<T>{y.x, y.y};
        vb[2 * h + 1] = Cx<T>{y.z, y.w};
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        vb[q] = (kb2 < K && nn0 + BQ * q < N) ? bbase[(size_t)kb2 * ldb + nn0 + BQ * q] : czero<T>();
    }
  };
  load(0);
  for (int kb = 0; kb < K; kb += GM_K) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *reinterpret_cast<Cx<T>*>(&sa[ar * SROW + 2 * (ak + q)]) = va[q];
      *reinterpret_cast<Cx<T>*>(&sb[(bn + BQ * q) * SROW + 2 * bk]) = vb[q];
    }
    __syncthreads();
    if (kb + GM_K < K) load(kb + GM_K);
    if constexpr (G3) {
      // lane (c16, kk) takes complex k = 4 st + kk: cre, cim, c3 accumulate t1, t2, t3
#pragma unroll
      for (int st = 0; st < GM_K / 4; ++st) {
        const int col = 2 * (4 * st + kk);
        T xr[2], xi[2], xs[2], yr[2], yi[2], ys[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const Cx<T> v = *reinterpret_cast<const Cx<T>*>(&sa[(wm + i * 16 + c16) * SROW + col]);
          xr[i] = v.re;
          xi[i] = v.im;
          xs[i] = v.re + v.im;
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const Cx<T> v = *reinterpret_cast<const Cx<T>*>(&sb[(wn + j * 16 + c16) * SROW + col]);
          yr[j] = v.re;
          yi[j] = v.im;
          ys[j] = v.re + v.im;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            cre[i][j] = MF::mma(xr[i], yr[j], cre[i][j]);
            cim[i][j] = MF::mma(xi[i], yi[j], cim[i][j]);
            c3[i][j] = MF::mma(xs[i], ys[j], c3[i][j]);
          }
      }
      __syncthreads();
      continue;
    }
#pragma unroll
    for (int st = 0; st < GM_K / 2; ++st) {
      const int col = 4 * st + kk;
      T av[2], bre[2], bim[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = sa[(wm + i * 16 + c16) * SROW + col];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const Cx<T> v = *reinterpret_cast<const Cx<T>*>(&sb[(wn + j * 16 + c16) * SROW + (col & ~1)]);
        bre[j] = (kk & 1) ? -v.im : v.re;
        bim[j] = (kk & 1) ? v.re : v.im;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cre[i][j] = MF::mma(av[i], bre[j], cre[i][j]);
          cim[i][j] = MF::mma(av[i], bim[j], cim[i][j]);
        }
    }
    __syncthreads();
  }
  if constexpr (G3) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const typename MF::acc t1 = cre[i][j], t2 = cim[i][j];
        cre[i][j] = t1 - t2;
        cim[i][j] = c3[i][j] - t1 - t2;
      }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm + i * 16 + MF::row(l, r);
      if (m >= M) continue;
      Cx<T>* crow = C + bt * sC + (size_t)(mapc ? mapc[m] : m) * ldc;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int nn = n0 + wn + j * 16 + c16;
        if (nn < N) {
          Cx<T> out{alpha * cre[i][j][r], alpha * cim[i][j][r]};
          if (beta != T(0)) out = out + beta * crow[nn];
          crow[nn] = out;
        }
      }
    }
}

// -------------------------------------------------------------- launchers
namespace {
unsigned grid1(size_t count, size_t cap = 8192) {
  size_t g = (count + 255) / 256;
  if (g > cap) g = cap;
  if (g == 0) g = 1;
  return (unsigned)g;
}
}  // namespace

template <typename T>
hipError_t launch_norm2(const Cx<T>* x, double* out, const int* vidx, int nvec, size_t n, hipStream_t s) {
  if (nvec <= 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(out, 0, sizeof(double) * nvec, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_norm2<T>), dim3(grid1(n, 256), nvec), dim3(256), 0, s, x, out, vidx, n);
  return hipGetLastError();
}

template <typename To, typename Ti>
hipError_t launch_convert(const Cx<Ti>* x, Cx<To>* y, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL((k_convert<To, Ti>), dim3(grid1(count)), dim3(256), 0, s, x, y, count);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_axpby(const Cx<T>* x, Cx<T>* y, double a, double b, const int* vidx, int nvec, size_t n,
                        hipStream_t s) {
  if (nvec <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_axpby<T>), dim3(grid1(n, 512), nvec), dim3(256), 0, s, x, y, (T)a, (T)b, vidx, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_accumulate(const Cx<T>* x, Cx<double>* y, double alpha, const int* vidx, int nvec, size_t n,
                             hipStream_t s) {
  if (nvec <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_accumulate<T>), dim3(grid1(n, 512), nvec), dim3(256), 0, s, x, y, alpha, vidx, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_real_to_complex(const double* in, Cx<T>* out, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL((k_real_to_complex<T>), dim3(grid1(count)), dim3(256), 0, s, in, out, count);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_philox_normal(Cx<T>* out, int nvec, size_t n, uint64_t seed, hipStream_t s, int k0) {
  if (nvec <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_philox_normal<T>), dim3(grid1((n + 1) / 2, 1024), nvec), dim3(256), 0, s, out, n, seed, k0);
  return hipGetLastError();
}

GemmPlan gemm_ah_b_plan(size_t n, size_t seg, int ksub) {
  GemmPlan p;
  if (seg == 0 || seg > n) seg = n;
  p.seg = seg;
  p.nseg = (int)((n + seg - 1) / seg);
  if (ksub < 1) ksub = 1;
  size_t chunk = (seg + ksub - 1) / ksub;
  p.chunk = (chunk + GM_K - 1) / GM_K * GM_K;
  p.ksub = (int)((seg + p.chunk - 1) / p.chunk);
  return p;
}

template <typename T>
hipError_t launch_gemm_ah_b_part(const Cx<T>* A, int na, const Cx<T>* B, const int* vidx, int nb, size_t n,
                                 const GemmPlan& p, Cx<double>* part, hipStream_t s, Cx<float>* out32) {
  if (na <= 0 || nb <= 0) return hipSuccess;
  if (out32 && p.ksub != 1) return hipErrorInvalidValue;
  if (nb <= 16) {  // one 16-wide b tile (see ah_b_body)
    dim3 grid((na + GM_T - 1) / GM_T, 1, (unsigned)(p.nseg * p.ksub));
    hipLaunchKernelGGL((k_gemm_ah_b_narrow<T>), grid, dim3(256), 0, s, A, na, B, vidx, nb, n, p.seg, p.chunk,
                       p.ksub, part, out32);
  } else {
    dim3 grid((na + GM_T - 1) / GM_T, (nb + GM_T - 1) / GM_T, (unsigned)(p.nseg * p.ksub));
    hipLaunchKernelGGL((k_gemm_ah_b_mfma<T>), grid, dim3(256), 0, s, A, na, B, vidx, nb, n, p.seg, p.chunk, p.ksub,
                       part, out32);
  }
  return hipGetLastError();
}

hipError_t launch_reduce_parts(const Cx<double>* part, const GemmPlan& p, size_t count, Cx<double>* C, double alpha,
                               hipStream_t s, Cx<float>* C32) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_parts, dim3(grid1(count * p.nseg, 2048)), dim3(256), 0, s, part, p.ksub, p.nseg, count,
                     C, alpha, C32);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm_ah_b_seg(const Cx<T>* A, int na, const Cx<T>* B, const int* vidx, int nb, size_t n, size_t seg,
                                Cx<double>* C, Cx<double>* part, int ksub, hipStream_t s, double alpha) {
  if (na <= 0 || nb <= 0) return hipSuccess;
  const GemmPlan p = gemm_ah_b_plan(n, seg, ksub);
  hipError_t e = launch_gemm_ah_b_part<T>(A, na, B, vidx, nb, n, p, part, s);
  if (e != hipSuccess) return e;
  return launch_reduce_parts(part, p, (size_t)na * nb, C, alpha, s);
}

template <typename T>
hipError_t launch_gemm_ah_b(const Cx<T>* A, int na, const Cx<T>* B, const int* vidx, int nb, size_t n,
                            Cx<double>* C, Cx<double>* part, int ksplit, hipStream_t s) {
  return launch_gemm_ah_b_seg<T>(A, na, B, vidx, nb, n, n, C, part, ksplit, s, 1.0);
}

template <typename T, typename MT>
hipError_t launch_gemm_update_seg(const Cx<T>* A, int na, const Cx<MT>* M, size_t mstride, int nb,
                                  const Cx<T>* X1, const Cx<T>* X2, double beta, Cx<T>* Y, const int* vidx, size_t n,
                                  size_t seg, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  // Y may be A itself when nb <= 64: then every workgroup covers all vectors of its k range in one pass and
  // reads all of that range's rows of A (before its last barrier) before it writes any of them
  if (static_cast<const void*>(Y) == static_cast<const void*>(A) && (nb > 64 || na != nb))
    return hipErrorInvalidValue;
  if (seg == 0 || seg >= n) {
    seg = n;
    mstride = 0;
  } else if (seg % 64 != 0) {
    return hipErrorInvalidValue;  // a workgroup's 64 elements must share one segment
  }
  const dim3 grid((unsigned)((n + 63) / 64));
  if (nb > 32) {
    if constexpr (sizeof(T) == 4) {
      const size_t tiles = ((n + UPD_T - 1) / UPD_T) * (size_t)((nb + UPD_T - 1) / UPD_T);
      hipLaunchKernelGGL((k_gemm_update_tile<MT>), dim3((unsigned)tiles), dim3(256), 0, s, A, na, M, nb, X1, X2,
                         (T)beta, Y, vidx, n, seg, mstride);
    } else
      hipLaunchKernelGGL((k_gemm_update_mfma<T, MT, 4, 4, 3>), grid, dim3(256), 0, s, A, na, M, nb, X1, X2, (T)beta,
                         Y, vidx, n, seg, mstride);
  } else if (nb > 16) {
    hipLaunchKernelGGL((k_gemm_update_mfma<T, MT, 2, 8, 0>), grid, dim3(256), 0, s, A, na, M, nb, X1, X2, (T)beta, Y,
                       vidx, n, seg, mstride);
  } else {  // one 16-wide b tile: a second one would run its MFMAs on zeros
    hipLaunchKernelGGL((k_gemm_update_mfma<T, MT, 1, 8, 0>), grid, dim3(256), 0, s, A, na, M, nb, X1, X2, (T)beta, Y,
                       vidx, n, seg, mstride);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm_update(const Cx<T>* A, int na, const Cx<double>* M, int nb, const Cx<T>* X1,
                              const Cx<T>* X2, double beta, Cx<T>* Y, const int* vidx, size_t n, hipStream_t s) {
  return launch_gemm_update_seg<T, double>(A, na, M, 0, nb, X1, X2, beta, Y, vidx, n, n, s);
}

hipError_t launch_gram_orth(const Cx<double>* G, Cx<double>* X, int na, double drop_tol, int* kept, hipStream_t s,
                            int batch, const double* gnorm) {
  if (batch <= 0) return hipSuccess;
  if (na < 1 || na > SMALL_NA) return hipErrorInvalidValue;  // callers orthonormalise in blocks of <= 64 columns
  hipLaunchKernelGGL(k_gram_orth_lds, dim3(batch), dim3(256), 0, s, G, X, na, drop_tol, kept, gnorm);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_seg_colnorm2(const Cx<T>* Y, int na, size_t n, size_t seg, int nseg, double* out, hipStream_t s) {
  if (na <= 0 || nseg <= 0) return hipSuccess;
  if (seg == 0 || (size_t)nseg * seg < n || (size_t)(nseg - 1) * seg >= n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_seg_colnorm2<T>, dim3((unsigned)(na * nseg)), dim3(256), 0, s, Y, na, n, seg, out);
  return hipGetLastError();
}
template hipError_t launch_seg_colnorm2<float>(const Cx<float>*, int, size_t, size_t, int, double*, hipStream_t);
template hipError_t launch_seg_colnorm2<double>(const Cx<double>*, int, size_t, size_t, int, double*, hipStream_t);

hipError_t launch_lu_inverse(const Cx<double>* M, size_t ldm, size_t sm, Cx<double>* Z, size_t ldz, size_t sz,
                             Cx<double>* work, int na, bool plain, int* singular, int batch, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if (na <= SMALL_NA)
    hipLaunchKernelGGL(k_lu_inverse_lds<double>, dim3(batch), dim3(256), 0, s, M, ldm, sm, Z, ldz, sz, na,
                       (int)plain, singular);
  else
    hipLaunchKernelGGL(k_lu_inverse_i_minus, dim3(batch), dim3(256), (sizeof(Cx<double>) + 2 * sizeof(int)) * na, s,
                       M, ldm, sm, Z, ldz, sz, work, na, (int)plain, singular);
  return hipGetLastError();
}

hipError_t launch_lu_inverse_small_f32(const Cx<float>* M, size_t ldm, size_t sm, Cx<float>* Z, size_t ldz, size_t sz,
                                      int na, bool plain, int* singular, int batch, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if (na < 1 || na > SMALL_NA) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lu_inverse_lds<float>, dim3(batch), dim3(256), 0, s, M, ldm, sm, Z, ldz, sz, na, (int)plain,
                     singular);
  return hipGetLastError();
}

hipError_t launch_lu_inverse_i_minus(const Cx<double>* M, Cx<double>* Z, Cx<double>* work, int na, int* singular,
                                     hipStream_t s) {
  return launch_lu_inverse(M, na, 0, Z, na, 0, work, na, false, singular, 1, s);
}

hipError_t launch_small_gemm(const Cx<double>* A, const Cx<double>* B, Cx<double>* C, int na, int nb, double alpha,
                             hipStream_t s, int batch) {
  if (batch <= 0 || na <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_small_gemm, dim3((na * nb + 255) / 256, batch), dim3(256), 0, s, A, B, C, na, nb, alpha);
  return hipGetLastError();
}

template <typename To>
hipError_t launch_leaf_form(const Cx<double>* ktab, const double* chi, Cx<To>* out, int nz, int nl, int leaf0,
                            int nleaf, hipStream_t s) {
  const size_t total = (size_t)nl * nl * nleaf;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL((k_leaf_form<To>), dim3(grid1(total, 16384)), dim3(256), 0, s, ktab, chi, out, nz, nl, leaf0,
                     nleaf);
  return hipGetLastError();
}
template hipError_t launch_leaf_form<double>(const Cx<double>*, const double*, Cx<double>*, int, int, int, int,
                                             hipStream_t);
template hipError_t launch_leaf_form<float>(const Cx<double>*, const double*, Cx<float>*, int, int, int, int,
                                            hipStream_t);

hipError_t launch_transpose_f32(const Cx<float>* in, Cx<float>* out, int m, int batch, hipStream_t s) {
  if (batch <= 0 || m <= 0) return hipSuccess;
  const dim3 grid((m + 31) / 32, (m + 31) / 32, batch);
  hipLaunchKernelGGL((k_transpose_convert<float, float>), grid, dim3(256), 0, s, in, out, m);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_transpose_convert(const Cx<double>* in, Cx<T>* out, int m, int batch, hipStream_t s) {
  if (batch <= 0 || m <= 0) return hipSuccess;
  const dim3 grid((m + 31) / 32, (m + 31) / 32, batch);
  hipLaunchKernelGGL((k_transpose_convert<T, double>), grid, dim3(256), 0, s, in, out, m);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bgemm(const Cx<T>* A, size_t lda, size_t sA, const Cx<T>* B, size_t ldb, size_t sB, Cx<T>* C,
                        size_t ldc, size_t sC, const int* mapa, const int* mapc, int M, int N, int K, double alpha,
                        double beta, int batch, hipStream_t s) {
  if (batch <= 0 || M <= 0 || N <= 0) return hipSuccess;
  const dim3 grid((N + GM_T - 1) / GM_T, (M + GM_T - 1) / GM_T, batch);
  hipLaunchKernelGGL((k_bgemm_mfma<T>), grid, dim3(256), 0, s, A, lda, sA, B, ldb, sB, C, ldc, sC, mapa, mapc, M, N,
                     K, (T)alpha, (T)beta);
  return hipGetLastError();
}

hipError_t launch_set_identity(Cx<double>* out, size_t ld, size_t st, int r, int batch, hipStream_t s) {
  const size_t total = (size_t)r * r * batch;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_identity, dim3(grid1(total, 8192)), dim3(256), 0, s, out, ld, st, r, batch);
  return hipGetLastError();
}

hipError_t launch_identity_deviation(const Cx<double>* P, size_t ld, size_t st, int r, int batch, double* dev,
                                     hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_identity_deviation, dim3(batch), dim3(256), 0, s, P, ld, st, r, dev);
  return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_f64, dim3(grid1(count, 1024)), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mask_slots(const Slot<T>* tab, const int* live, int nslots, size_t n, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_mask_slots<T>), dim3(grid1(n, 256), nslots), dim3(256), 0, s, tab, live, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_axpy_map(const Cx<T>* x, Cx<T>* y, const int* yidx, double a, int nvec, size_t n, hipStream_t s) {
  if (nvec <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_axpy_map<T>), dim3(grid1(n, 512), nvec), dim3(256), 0, s, x, y, yidx, (T)a, n);
  return hipGetLastError();
}

#define LSOP_INST_LA(T)                                                                                              \
  template hipError_t launch_norm2<T>(const Cx<T>*, double*, const int*, int, size_t, hipStream_t);                 \
  template hipError_t launch_axpby<T>(const Cx<T>*, Cx<T>*, double, double, const int*, int, size_t, hipStream_t);  \
  template hipError_t launch_accumulate<T>(const Cx<T>*, Cx<double>*, double, const int*, int, size_t,          \
                                           hipStream_t);        \
  template hipError_t launch_real_to_complex<T>(const double*, Cx<T>*, size_t, hipStream_t);                        \
  template hipError_t launch_philox_normal<T>(Cx<T>*, int, size_t, uint64_t, hipStream_t, int);                     \
  template hipError_t launch_gemm_ah_b<T>(const Cx<T>*, int, const Cx<T>*, const int*, int, size_t, Cx<double>*,    \
                                          Cx<double>*, int, hipStream_t);                                           \
  template hipError_t launch_gemm_ah_b_seg<T>(const Cx<T>*, int, const Cx<T>*, const int*, int, size_t, size_t,     \
                                              Cx<double>*, Cx<double>*, int, hipStream_t, double);                  \
  template hipError_t launch_gemm_ah_b_part<T>(const Cx<T>*, int, const Cx<T>*, const int*, int, size_t,            \
                                               const GemmPlan&, Cx<double>*, hipStream_t, Cx<float>*);              \
  template hipError_t launch_gemm_update<T>(const Cx<T>*, int, const Cx<double>*, int, const Cx<T>*, const Cx<T>*, \
                                            double, Cx<T>*, const int*, size_t, hipStream_t);                       \
  template hipError_t launch_gemm_update_seg<T, double>(const Cx<T>*, int, const Cx<double>*, size_t, int,       \
                                                        const Cx<T>*, const Cx<T>*, double, Cx<T>*, const int*,    \
                                                        size_t, size_t, hipStream_t);                               \
  template hipError_t launch_transpose_convert<T>(const Cx<double>*, Cx<T>*, int, int, hipStream_t);               \
  template hipError_t launch_bgemm<T>(const Cx<T>*, size_t, size_t, const Cx<T>*, size_t, size_t, Cx<T>*, size_t,  \
                                      size_t, const int*, const int*, int, int, int, double, double, int,          \
                                      hipStream_t);                                                                 \
  template hipError_t launch_axpy_map<T>(const Cx<T>*, Cx<T>*, const int*, double, int, size_t, hipStream_t);       \
  template hipError_t launch_mask_slots<T>(const Slot<T>*, const int*, int, size_t, hipStream_t);
LSOP_INST_LA(float)
LSOP_INST_LA(double)
template hipError_t launch_gemm_update_seg<float, float>(const Cx<float>*, int, const Cx<float>*, size_t, int,
                                                         const Cx<float>*, const Cx<float>*, double, Cx<float>*,
                                                         const int*, size_t, size_t, hipStream_t);
template hipError_t launch_convert<float, double>(const Cx<double>*, Cx<float>*, size_t, hipStream_t);
template hipError_t launch_convert<double, float>(const Cx<float>*, Cx<double>*, size_t, hipStream_t);

}  // namespace lsop
