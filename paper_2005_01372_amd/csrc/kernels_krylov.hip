// Vector kernels of the restarted GMRES solver (the Krylov comparison method
// of the paper's Section 3.2.3), batched over right-hand sides.
//
// The Krylov basis is stored [basis vector i][right-hand side s][n]: basis
// vector i of every right-hand side is one [nvec][n] block, addressed like the
// series' vectors through the active list vidx.  All sums are FP64.
#include "internal.hpp"

namespace lsop {

namespace {
constexpr int kThreads = 256;
constexpr int kPerThread = 4;                       // elements of one vector per thread and chunk
constexpr int kChunk = kThreads * kPerThread;      // elements per workgroup

__device__ __forceinline__ double2 block_sum2(double2 v, double2* red) {
  // sum of one (re, im) pair over the workgroup; red: kThreads / 64 slots; result valid in every thread
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    s.x += red[w].x;
    s.y += red[w].y;
  }
  return s;
}
}  // namespace

// part[((a * nb) + i) * nchunk + c] = sum over chunk c of conj(V[i][vs][k]) w[vs][k], vs = vidx[a]
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mdot(const Cx<T>* __restrict__ V, size_t bstride, int nb,
                                                   const Cx<T>* __restrict__ w, const int* __restrict__ vidx,
                                                   size_t n, int nchunk, Cx<double>* __restrict__ part) {
  __shared__ double2 red[kThreads / 64];
  const int a = blockIdx.y, c = blockIdx.x;
  const size_t vs = (size_t)vidx[a];
  const size_t k0 = (size_t)c * kChunk + threadIdx.x;
  Cx<T> wv[kPerThread];
#pragma unroll
  for (int e = 0; e < kPerThread; ++e) {
    const size_t k = k0 + (size_t)e * kThreads;
    wv[e] = k < n ? w[vs * n + k] : czero<T>();
  }
  for (int i = 0; i < nb; ++i) {
    const Cx<T>* vi = V + (size_t)i * bstride + vs * n;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int e = 0; e < kPerThread; ++e) {
      const size_t k = k0 + (size_t)e * kThreads;
      if (k < n) {
        const Cx<T> x = vi[k];
        acc.x += (double)x.re * (double)wv[e].re + (double)x.im * (double)wv[e].im;
        acc.y += (double)x.re * (double)wv[e].im - (double)x.im * (double)wv[e].re;
      }
    }
    const double2 s = block_sum2(acc, red);
    if (threadIdx.x == 0) part[((size_t)a * nb + i) * nchunk + c] = Cx<double>{s.x, s.y};
  }
}

// h[a * hstride + i] (+)= sum_c part[((a * nb) + i) * nchunk + c]  (one thread per (a, i))
__global__ void k_mdot_reduce(const Cx<double>* __restrict__ part, int na, int nb, int nchunk,
                              Cx<double>* __restrict__ h, int hstride, int accumulate) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= na * nb) return;
  const int a = t / nb, i = t % nb;
  double re = 0.0, im = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    const Cx<double> v = part[((size_t)a * nb + i) * nchunk + c];
    re += v.re;
    im += v.im;
  }
  Cx<double>& o = h[(size_t)a * hstride + i];
  if (accumulate) o = Cx<double>{o.re + re, o.im + im};
  else o = Cx<double>{re, im};
}

// out[vs] = beta * out[vs] + alpha * sum_{i < nb} coef[a * cstride + i] V[i][vs]   (vs = vidx[a]; beta = 0:
// out is not read)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mcombine(const Cx<T>* __restrict__ V, size_t bstride, int nb,
                                                       const Cx<double>* __restrict__ coef, int cstride,
                                                       double alpha, double beta, Cx<T>* __restrict__ out,
                                                       const int* __restrict__ vidx, size_t n) {
  const int a = blockIdx.y;
  const size_t vs = (size_t)vidx[a];
  const Cx<double>* ca = coef + (size_t)a * cstride;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    double re = 0.0, im = 0.0;
    if (beta != 0.0) {
      const Cx<T> o = out[vs * n + k];
      re = beta * (double)o.re;
      im = beta * (double)o.im;
    }
    double sr = 0.0, si = 0.0;
    for (int i = 0; i < nb; ++i) {
      const Cx<T> x = V[(size_t)i * bstride + vs * n + k];
      const Cx<double> cf = ca[i];
      sr += cf.re * (double)x.re - cf.im * (double)x.im;
      si += cf.re * (double)x.im + cf.im * (double)x.re;
    }
    re += alpha * sr;
    im += alpha * si;
    out[vs * n + k] = Cx<T>{(T)re, (T)im};
  }
}

// y[vs] = (sign / sqrt(nrm2[a])) x[vs], or 0 where nrm2[a] == 0 (a breakdown: the vector is already in the span)
template <typename T>
__global__ void k_scale_by_norm(const Cx<T>* __restrict__ x, Cx<T>* __restrict__ y, const double* __restrict__ nrm2,
                                double sign, const int* __restrict__ vidx, size_t n) {
  const int a = blockIdx.y;
  const size_t vs = (size_t)vidx[a];
  const double nr = nrm2[a];
  const T f = nr > 0.0 ? (T)(sign / sqrt(nr)) : T(0);
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const Cx<T> v = x[vs * n + k];
    y[vs * n + k] = Cx<T>{f * v.re, f * v.im};
  }
}

namespace {
int grid_x(size_t n) {
  const size_t b = (n + kThreads - 1) / kThreads;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}
}  // namespace

int mdot_chunks(size_t n) { return (int)((n + kChunk - 1) / kChunk); }

template <typename T>
hipError_t launch_mdot(const Cx<T>* V, size_t bstride, int nb, const Cx<T>* w, const int* vidx, int na, size_t n,
                       Cx<double>* part, Cx<double>* h, int hstride, bool accumulate, hipStream_t s) {
  if (na <= 0 || nb <= 0) return hipSuccess;
  const int nchunk = mdot_chunks(n);
  hipLaunchKernelGGL((k_mdot<T>), dim3(nchunk, na), dim3(kThreads), 0, s, V, bstride, nb, w, vidx, n, nchunk, part);
  const int tot = na * nb;
  hipLaunchKernelGGL(k_mdot_reduce, dim3((tot + 127) / 128), dim3(128), 0, s, part, na, nb, nchunk, h, hstride,
                     (int)accumulate);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mcombine(const Cx<T>* V, size_t bstride, int nb, const Cx<double>* coef, int cstride, double alpha,
                           double beta, Cx<T>* out, const int* vidx, int na, size_t n, hipStream_t s) {
  if (na <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_mcombine<T>), dim3(grid_x(n), na), dim3(kThreads), 0, s, V, bstride, nb, coef, cstride, alpha,
                     beta, out, vidx, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_by_norm(const Cx<T>* x, Cx<T>* y, const double* nrm2, double sign, const int* vidx, int na,
                                size_t n, hipStream_t s) {
  if (na <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_scale_by_norm<T>), dim3(grid_x(n), na), dim3(kThreads), 0, s, x, y, nrm2, sign, vidx, n);
  return hipGetLastError();
}

#define LSOP_INST_KRYLOV(T)                                                                                     \
  template hipError_t launch_mdot<T>(const Cx<T>*, size_t, int, const Cx<T>*, const int*, int, size_t,        \
                                     Cx<double>*, Cx<double>*, int, bool, hipStream_t);                        \
  template hipError_t launch_mcombine<T>(const Cx<T>*, size_t, int, const Cx<double>*, int, double, double,    \
                                         Cx<T>*, const int*, int, size_t, hipStream_t);                        \
  template hipError_t launch_scale_by_norm<T>(const Cx<T>*, Cx<T>*, const double*, double, const int*, int,    \
                                              size_t, hipStream_t);
LSOP_INST_KRYLOV(float)
LSOP_INST_KRYLOV(double)

}  // namespace lsop
