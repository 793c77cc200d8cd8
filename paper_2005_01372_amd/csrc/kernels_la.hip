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

template <typename T>
__global__ void k_axpby(const Cx<T>* __restrict__ x, Cx<T>* __restrict__ y, T a, T b, const int* __restrict__ vidx,
                        size_t n) {
  const int slot = blockIdx.y;
  const size_t off = (size_t)(vidx ? vidx[slot] : slot) * n;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const Cx<T> xv = x[off + k];
    const Cx<T> yv = y[off + k];
    y[off + k] = Cx<T>{a * xv.re + b * yv.re, a * xv.im + b * yv.im};
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
__global__ void k_philox_normal(Cx<T>* __restrict__ out, size_t n, uint64_t seed) {
  const int k = blockIdx.y;
  const size_t npairs = (n + 1) / 2;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < npairs; t += (size_t)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)(t & 0xffffffffu), (uint32_t)(t >> 32), (uint32_t)k, 0u};
    philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    const double u1 = ((double)c[0] + 0.5) * 2.3283064365386962890625e-10;
    const double u2 = ((double)c[1] + 0.5) * 2.3283064365386962890625e-10;
    const double r = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    Cx<T>* o = out + (size_t)k * n;
    o[2 * t] = Cx<T>{(T)(r * cs), T(0)};
    if (2 * t + 1 < n) o[2 * t + 1] = Cx<T>{(T)(r * sn), T(0)};
  }
}

// ---------------------------------------------------------- C = A^H B (split over n)
constexpr int GA_T = 32;   // output tile (a and b)
constexpr int GA_K = 32;   // k step staged in LDS

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_ah_b(const Cx<T>* __restrict__ A, int na, const Cx<T>* __restrict__ B,
                                                    const int* __restrict__ vidx, int nb, size_t n, size_t chunk,
                                                    Cx<double>* __restrict__ part) {
  __shared__ Cx<T> sa[GA_T][GA_K + 1];
  __shared__ Cx<T> sb[GA_T][GA_K + 1];
  const int a0 = blockIdx.x * GA_T, b0 = blockIdx.y * GA_T, ks = blockIdx.z;
  const size_t k_begin = (size_t)ks * chunk;
  const size_t k_end = k_begin + chunk < n ? k_begin + chunk : n;
  const int ta = (threadIdx.x / 16) * 2, tb = (threadIdx.x % 16) * 2;
  Cx<double> acc[2][2] = {};
  for (size_t kk = k_begin; kk < k_end; kk += GA_K) {
    for (int idx = threadIdx.x; idx < GA_T * GA_K; idx += 256) {
      const int r = idx / GA_K, c = idx % GA_K;
      const size_t k = kk + c;
      const bool kin = k < k_end;
      sa[r][c] = (kin && a0 + r < na) ? A[(size_t)(a0 + r) * n + k] : czero<T>();
      int vb = b0 + r;
      sb[r][c] = (kin && vb < nb) ? B[(size_t)(vidx ? vidx[vb] : vb) * n + k] : czero<T>();
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < GA_K; ++c) {
      const Cx<double> x0 = ccast<double>(sa[ta][c]), x1 = ccast<double>(sa[ta + 1][c]);
      const Cx<double> y0 = ccast<double>(sb[tb][c]), y1 = ccast<double>(sb[tb + 1][c]);
      acc[0][0] = acc[0][0] + cmul_conj(x0, y0);
      acc[0][1] = acc[0][1] + cmul_conj(x0, y1);
      acc[1][0] = acc[1][0] + cmul_conj(x1, y0);
      acc[1][1] = acc[1][1] + cmul_conj(x1, y1);
    }
    __syncthreads();
  }
  Cx<double>* p = part + (size_t)ks * na * nb;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if (a0 + ta + i < na && b0 + tb + j < nb) p[(size_t)(a0 + ta + i) * nb + b0 + tb + j] = acc[i][j];
}

__global__ void k_reduce_parts(const Cx<double>* __restrict__ part, int nparts, size_t count,
                               Cx<double>* __restrict__ C) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x) {
    Cx<double> s = czero<double>();
    for (int p = 0; p < nparts; ++p) s = s + part[(size_t)p * count + k];
    C[k] = s;
  }
}

// ---------------------------------------------------------- Y = X1 + beta X2 + A M
constexpr int GU_B = 16;  // b columns per pass
constexpr int GU_A = 16;  // a rows per register block

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_update(const Cx<T>* __restrict__ A, int na,
                                                      const Cx<double>* __restrict__ M, int nb,
                                                      const Cx<T>* X1, const Cx<T>* X2, T beta, Cx<T>* Y,
                                                      const int* __restrict__ vidx, size_t n) {
  extern __shared__ unsigned char smem_raw[];
  Cx<T>* sm = reinterpret_cast<Cx<T>*>(smem_raw);  // [na][GU_B]
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool kin = k < n;
  for (int b0 = 0; b0 < nb; b0 += GU_B) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < na * GU_B; idx += blockDim.x) {
      const int a = idx / GU_B, bb = idx % GU_B;
      sm[idx] = (b0 + bb < nb) ? ccast<T>(M[(size_t)a * nb + b0 + bb]) : czero<T>();
    }
    __syncthreads();
    Cx<T> acc[GU_B];
#pragma unroll
    for (int bb = 0; bb < GU_B; ++bb) acc[bb] = czero<T>();
    for (int a0 = 0; a0 < na; a0 += GU_A) {
      Cx<T> av[GU_A];
#pragma unroll
      for (int j = 0; j < GU_A; ++j) av[j] = (kin && a0 + j < na) ? A[(size_t)(a0 + j) * n + k] : czero<T>();
#pragma unroll
      for (int j = 0; j < GU_A; ++j) {
        if (a0 + j < na) {
#pragma unroll
          for (int bb = 0; bb < GU_B; ++bb) acc[bb] = acc[bb] + av[j] * sm[(a0 + j) * GU_B + bb];
        }
      }
    }
    if (kin) {
#pragma unroll
      for (int bb = 0; bb < GU_B; ++bb) {
        const int b = b0 + bb;
        if (b < nb) {
          const size_t off = (size_t)(vidx ? vidx[b] : b) * n + k;
          Cx<T> out = acc[bb];
          if (X1) out = out + X1[off];
          if (X2) out = out + beta * X2[off];
          Y[off] = out;
        }
      }
    }
  }
}

// ------------------------------------------------------- small FP64 kernels
// Orthonormalising coefficients X (na x na) for Q = Y X from the Gram matrix
// G = Y^H Y: column k of X is e_k projected twice (classical Gram-Schmidt in
// the G inner product) against the kept columns, then normalised; columns
// whose remaining G-norm^2 is <= drop_tol * G_kk are zeroed (dropped).
// G and X point to LDS copies (na <= SMALL_NA) or to global memory.
constexpr int SMALL_NA = 64;

__device__ __forceinline__ void gram_orth_body(const Cx<double>* G, Cx<double>* X, int na, double drop_tol,
                                               Cx<double>* x, Cx<double>* w, Cx<double>* cf, double* red,
                                               int* nkept_out) {
  const int t = threadIdx.x;
  for (int i = t; i < na * na; i += blockDim.x) X[i] = czero<double>();
  __syncthreads();
  int nkept = 0;
  for (int k = 0; k < na; ++k) {
    for (int i = t; i < na; i += blockDim.x) x[i] = Cx<double>{i == k ? 1.0 : 0.0, 0.0};
    __syncthreads();
    for (int pass = 0; pass < 3; ++pass) {
      // w = G x
      for (int i = t; i < na; i += blockDim.x) {
        Cx<double> s = czero<double>();
        for (int l = 0; l < na; ++l) s = s + G[(size_t)i * na + l] * x[l];
        w[i] = s;
      }
      __syncthreads();
      if (pass == 2) break;
      // cf_j = X[:, j]^H w for j < k
      for (int j = t; j < k; j += blockDim.x) {
        Cx<double> s = czero<double>();
        for (int i = 0; i < na; ++i) s = s + cmul_conj(X[(size_t)i * na + j], w[i]);
        cf[j] = s;
      }
      __syncthreads();
      // x -= X[:, :k] cf
      for (int i = t; i < na; i += blockDim.x) {
        Cx<double> s = czero<double>();
        for (int j = 0; j < k; ++j) s = s + X[(size_t)i * na + j] * cf[j];
        x[i] = x[i] - s;
      }
      __syncthreads();
    }
    // nrm2 = x^H G x = x^H w
    double part = 0.0;
    for (int i = t; i < na; i += blockDim.x) part += x[i].re * w[i].re + x[i].im * w[i].im;
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if ((t & 63) == 0) red[t >> 6] = part;
    __syncthreads();
    double nrm2 = 0.0;
    for (int i = 0; i < (int)(blockDim.x / 64); ++i) nrm2 += red[i];
    const double gkk = G[(size_t)k * na + k].re;
    const bool keep = gkk > 1e-300 && nrm2 > drop_tol * gkk;
    const double sc = keep ? 1.0 / sqrt(nrm2) : 0.0;
    for (int i = t; i < na; i += blockDim.x) X[(size_t)i * na + k] = sc * x[i];
    nkept += keep ? 1 : 0;
    __syncthreads();
  }
  *nkept_out = nkept;
}

__global__ __launch_bounds__(256) void k_gram_orth_lds(const Cx<double>* __restrict__ Gg, Cx<double>* __restrict__ Xg,
                                                        int na, double drop_tol, int* kept) {
  __shared__ Cx<double> G[SMALL_NA * SMALL_NA], X[SMALL_NA * SMALL_NA];
  __shared__ Cx<double> x[SMALL_NA], w[SMALL_NA], cf[SMALL_NA];
  __shared__ double red[4];
  for (int i = threadIdx.x; i < na * na; i += blockDim.x) G[i] = Gg[i];
  __syncthreads();
  int nk = 0;
  gram_orth_body(G, X, na, drop_tol, x, w, cf, red, &nk);
  for (int i = threadIdx.x; i < na * na; i += blockDim.x) Xg[i] = X[i];
  if (threadIdx.x == 0) *kept = nk;
}

__global__ __launch_bounds__(256) void k_gram_orth(const Cx<double>* __restrict__ G, Cx<double>* __restrict__ X,
                                                    int na, double drop_tol, int* kept) {
  extern __shared__ unsigned char smem_raw[];
  Cx<double>* x = reinterpret_cast<Cx<double>*>(smem_raw);  // [na]
  Cx<double>* w = x + na;                                    // [na] = G x
  Cx<double>* cf = w + na;                                   // [na] projections
  __shared__ double red[4];
  int nk = 0;
  gram_orth_body(G, X, na, drop_tol, x, w, cf, red, &nk);
  if (threadIdx.x == 0) *kept = nk;
}

// Z = (I - M)^{-1}, Gauss-Jordan with partial pivoting on work = [I - M | I]
// (work in LDS for na <= SMALL_NA, else in global memory).
__device__ __forceinline__ void lu_inverse_body(const Cx<double>* M, Cx<double>* Z, Cx<double>* work, int na,
                                                int* singular, Cx<double>* fcol, double* best, int* bidx,
                                                double* scale_s) {
  const int t = threadIdx.x, w2 = 2 * na;
  double amax = 0.0;
  for (int idx = t; idx < na * w2; idx += blockDim.x) {
    const int i = idx / w2, j = idx % w2;
    Cx<double> v;
    if (j < na) v = Cx<double>{(i == j ? 1.0 : 0.0) - M[(size_t)i * na + j].re, -M[(size_t)i * na + j].im};
    else v = Cx<double>{(i == j - na) ? 1.0 : 0.0, 0.0};
    work[idx] = v;
    if (j < na) amax = fmax(amax, sqrt(norm2(v)));
  }
  best[t] = amax;
  __syncthreads();
  if (t == 0) {
    double m = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) m = fmax(m, best[i]);
    *scale_s = m;
    *singular = 0;
  }
  __syncthreads();
  const double scale = *scale_s;
  for (int k = 0; k < na; ++k) {
    double bv = -1.0;
    int bi = k;
    for (int i = k + t; i < na; i += blockDim.x) {
      const double v = norm2(work[(size_t)i * w2 + k]);
      if (v > bv) {
        bv = v;
        bi = i;
      }
    }
    best[t] = bv;
    bidx[t] = bi;
    __syncthreads();
    if (t == 0) {
      double m = -1.0;
      int mi = k;
      for (int i = 0; i < (int)blockDim.x; ++i)
        if (best[i] > m) {
          m = best[i];
          mi = bidx[i];
        }
      bidx[0] = mi;
      best[0] = m;
    }
    __syncthreads();
    const int p = bidx[0];
    const double piv2 = best[0];
    if (!(sqrt(piv2) > 1e-14 * scale)) {
      if (t == 0) *singular = 1;
      return;  // uniform across the workgroup
    }
    if (p != k) {
      for (int j = t; j < w2; j += blockDim.x) {
        const Cx<double> a = work[(size_t)k * w2 + j];
        work[(size_t)k * w2 + j] = work[(size_t)p * w2 + j];
        work[(size_t)p * w2 + j] = a;
      }
    }
    __syncthreads();
    const Cx<double> pv = work[(size_t)k * w2 + k];
    const double d = 1.0 / norm2(pv);
    const Cx<double> inv = Cx<double>{pv.re * d, -pv.im * d};
    __syncthreads();
    for (int j = t; j < w2; j += blockDim.x) work[(size_t)k * w2 + j] = work[(size_t)k * w2 + j] * inv;
    for (int i = t; i < na; i += blockDim.x) fcol[i] = work[(size_t)i * w2 + k];
    __syncthreads();
    for (int idx = t; idx < na * w2; idx += blockDim.x) {
      const int i = idx / w2, j = idx % w2;
      if (i != k) work[idx] = work[idx] - fcol[i] * work[(size_t)k * w2 + j];
    }
    __syncthreads();
  }
  for (int idx = t; idx < na * na; idx += blockDim.x) {
    const int i = idx / na, j = idx % na;
    Z[idx] = work[(size_t)i * w2 + na + j];
  }
}

__global__ __launch_bounds__(256) void k_lu_inverse_lds(const Cx<double>* __restrict__ M, Cx<double>* __restrict__ Z,
                                                         int na, int* singular) {
  __shared__ Cx<double> work[SMALL_NA * 2 * SMALL_NA];
  __shared__ Cx<double> fcol[SMALL_NA];
  __shared__ double best[256];
  __shared__ int bidx[256];
  __shared__ double scale;
  lu_inverse_body(M, Z, work, na, singular, fcol, best, bidx, &scale);
}

__global__ __launch_bounds__(256) void k_lu_inverse_i_minus(const Cx<double>* __restrict__ M,
                                                             Cx<double>* __restrict__ Z, Cx<double>* __restrict__ work,
                                                             int na, int* singular) {
  extern __shared__ unsigned char smem_raw[];
  Cx<double>* fcol = reinterpret_cast<Cx<double>*>(smem_raw);  // [na]
  __shared__ double best[256];
  __shared__ int bidx[256];
  __shared__ double scale;
  lu_inverse_body(M, Z, work, na, singular, fcol, best, bidx, &scale);
}

__global__ void k_small_gemm(const Cx<double>* __restrict__ A, const Cx<double>* __restrict__ B,
                             Cx<double>* __restrict__ C, int na, int nb, double alpha) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= na * nb) return;
  const int i = idx / nb, j = idx % nb;
  Cx<double> s = czero<double>();
  for (int l = 0; l < na; ++l) s = s + A[(size_t)i * na + l] * B[(size_t)l * nb + j];
  C[idx] = alpha * s;
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
hipError_t launch_philox_normal(Cx<T>* out, int nvec, size_t n, uint64_t seed, hipStream_t s) {
  if (nvec <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_philox_normal<T>), dim3(grid1((n + 1) / 2, 1024), nvec), dim3(256), 0, s, out, n, seed);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm_ah_b(const Cx<T>* A, int na, const Cx<T>* B, const int* vidx, int nb, size_t n,
                            Cx<double>* C, Cx<double>* part, int ksplit, hipStream_t s) {
  if (na <= 0 || nb <= 0) return hipSuccess;
  size_t chunk = (n + ksplit - 1) / ksplit;
  chunk = (chunk + GA_K - 1) / GA_K * GA_K;
  const int parts = (int)((n + chunk - 1) / chunk);
  dim3 grid((na + GA_T - 1) / GA_T, (nb + GA_T - 1) / GA_T, parts);
  hipLaunchKernelGGL((k_gemm_ah_b<T>), grid, dim3(256), 0, s, A, na, B, vidx, nb, n, chunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_parts, dim3(grid1((size_t)na * nb, 64)), dim3(256), 0, s, part, parts,
                     (size_t)na * nb, C);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm_update(const Cx<T>* A, int na, const Cx<double>* M, int nb, const Cx<T>* X1,
                              const Cx<T>* X2, double beta, Cx<T>* Y, const int* vidx, size_t n, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  const size_t shm = sizeof(Cx<T>) * (size_t)na * GU_B;
  hipLaunchKernelGGL((k_gemm_update<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), shm, s, A, na, M, nb, X1, X2,
                     (T)beta, Y, vidx, n);
  return hipGetLastError();
}

hipError_t launch_gram_orth(const Cx<double>* G, Cx<double>* X, int na, double drop_tol, int* kept,
                            hipStream_t s) {
  if (na <= SMALL_NA)
    hipLaunchKernelGGL(k_gram_orth_lds, dim3(1), dim3(256), 0, s, G, X, na, drop_tol, kept);
  else
    hipLaunchKernelGGL(k_gram_orth, dim3(1), dim3(256), sizeof(Cx<double>) * 3 * na, s, G, X, na, drop_tol, kept);
  return hipGetLastError();
}

hipError_t launch_lu_inverse_i_minus(const Cx<double>* M, Cx<double>* Z, Cx<double>* work, int na, int* singular,
                                     hipStream_t s) {
  if (na <= SMALL_NA)
    hipLaunchKernelGGL(k_lu_inverse_lds, dim3(1), dim3(256), 0, s, M, Z, na, singular);
  else
    hipLaunchKernelGGL(k_lu_inverse_i_minus, dim3(1), dim3(256), sizeof(Cx<double>) * na, s, M, Z, work, na,
                       singular);
  return hipGetLastError();
}

hipError_t launch_small_gemm(const Cx<double>* A, const Cx<double>* B, Cx<double>* C, int na, int nb, double alpha,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_small_gemm, dim3(grid1((size_t)na * nb)), dim3(256), 0, s, A, B, C, na, nb, alpha);
  return hipGetLastError();
}

#define LSOP_INST_LA(T)                                                                                              \
  template hipError_t launch_norm2<T>(const Cx<T>*, double*, const int*, int, size_t, hipStream_t);                 \
  template hipError_t launch_axpby<T>(const Cx<T>*, Cx<T>*, double, double, const int*, int, size_t, hipStream_t);  \
  template hipError_t launch_accumulate<T>(const Cx<T>*, Cx<double>*, double, const int*, int, size_t,          \
                                           hipStream_t);        \
  template hipError_t launch_real_to_complex<T>(const double*, Cx<T>*, size_t, hipStream_t);                        \
  template hipError_t launch_philox_normal<T>(Cx<T>*, int, size_t, uint64_t, hipStream_t);                          \
  template hipError_t launch_gemm_ah_b<T>(const Cx<T>*, int, const Cx<T>*, const int*, int, size_t, Cx<double>*,    \
                                          Cx<double>*, int, hipStream_t);                                           \
  template hipError_t launch_gemm_update<T>(const Cx<T>*, int, const Cx<double>*, int, const Cx<T>*, const Cx<T>*, \
                                            double, Cx<T>*, const int*, size_t, hipStream_t);
LSOP_INST_LA(float)
LSOP_INST_LA(double)
template hipError_t launch_convert<float, double>(const Cx<double>*, Cx<float>*, size_t, hipStream_t);
template hipError_t launch_convert<double, float>(const Cx<float>*, Cx<double>*, size_t, hipStream_t);

}  // namespace lsop
