// Kernels of the convergent Born series (Section 2.2's review of the series with a dissipative background):
// the kernel table at complex wavenumber, the complex potential V_eps = chi - i eps r with its absorbing-layer
// profile r, the pointwise products with V_eps around the FFT convolution, and H = gamma = i V_eps / eps.
#include "bessel_complex.hpp"
#include "internal.hpp"

namespace lsop {

// K(p,q) = cj1 H0^(1)(kh rho), rho = sqrt(p^2 + q^2) > 0; K(0,0) = self (complex kh)
__global__ void k_table_c(Cx<double>* __restrict__ ktab, int nx, int nz, Cx<double> kh, Cx<double> cj1,
                          Cx<double> self) {
  const int n = nx * nz;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int p = k / nz, q = k % nz;
    if (p == 0 && q == 0) {
      ktab[k] = self;
      continue;
    }
    const double rho = sqrt((double)(p * p + q * q));
    ktab[k] = cj1 * lsop_bessel::hankel0_c(rho * kh);
  }
}

// V_eps = chi - i eps r(d), r = 1 - max(0, 1 - d / absorb) / 2 with d the distance of the cell to the grid edge
// (in cells); absorb = 0: r = 1
__global__ void k_damped_potential(const double* __restrict__ chi, int nx, int nz, double eps, int absorb,
                                   Cx<double>* __restrict__ v64, Cx<float>* __restrict__ v32) {
  const int n = nx * nz;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int i = k / nz, j = k % nz;
    double r = 1.0;
    if (absorb > 0) {
      const int d = min(min(i, j), min(nx - 1 - i, nz - 1 - j));
      r = 1.0 - 0.5 * fmax(0.0, 1.0 - (double)d / absorb);
    }
    const Cx<double> v{chi[k], -eps * r};
    if (v64) v64[k] = v;
    if (v32) v32[k] = ccast<float>(v);
  }
}

// Pointwise products with the complex potential over nvec vectors; x is addressed through xidx, y through yidx
// (NULL: slot order), c is compact ([slot][n]):
//  op 0: y = V x;  op 1: y = x - conj(V) c;  op 2: y = conj(V) c;
//  op 3: y = gamma x;  op 4: y = y - gamma x   (gamma = i V / eps, scale = 1 / eps)
template <typename T>
__global__ void k_vmul(const Cx<T>* __restrict__ V, const Cx<T>* x, const int* __restrict__ xidx, const Cx<T>* c,
                       Cx<T>* y, const int* __restrict__ yidx, size_t n, int op, T scale) {
  const int slot = blockIdx.y;
  const size_t ox = (size_t)(xidx ? xidx[slot] : slot) * n;
  const size_t oy = (size_t)(yidx ? yidx[slot] : slot) * n;
  const size_t oc = (size_t)slot * n;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const Cx<T> v = V[k];
    const Cx<T> g{-scale * v.im, scale * v.re};
    Cx<T> out;
    switch (op) {
      case 0: out = v * x[ox + k]; break;
      case 1: out = x[ox + k] - cmul_conj(v, c[oc + k]); break;
      case 2: out = cmul_conj(v, c[oc + k]); break;
      case 3: out = g * x[ox + k]; break;
      default: out = y[oy + k] - g * x[ox + k]; break;
    }
    y[oy + k] = out;
  }
}

hipError_t launch_table_c(Cx<double>* ktab, int nx, int nz, Cx<double> kh, Cx<double> cj1, Cx<double> self,
                          hipStream_t s) {
  const int n = nx * nz;
  int grid = (n + 255) / 256;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_table_c, dim3(grid), dim3(256), 0, s, ktab, nx, nz, kh, cj1, self);
  return hipGetLastError();
}

hipError_t launch_damped_potential(const double* chi, int nx, int nz, double eps, int absorb, Cx<double>* v64,
                                   Cx<float>* v32, hipStream_t s) {
  const int n = nx * nz;
  int grid = (n + 255) / 256;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_damped_potential, dim3(grid), dim3(256), 0, s, chi, nx, nz, eps, absorb, v64, v32);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_vmul(const Cx<T>* V, const Cx<T>* x, const int* xidx, const Cx<T>* c, Cx<T>* y, const int* yidx,
                       int nvec, size_t n, int op, double scale, hipStream_t s) {
  if (nvec <= 0) return hipSuccess;
  size_t g = (n + 255) / 256;
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL((k_vmul<T>), dim3((unsigned)g, nvec), dim3(256), 0, s, V, x, xidx, c, y, yidx, n, op,
                     (T)scale);
  return hipGetLastError();
}

template hipError_t launch_vmul<float>(const Cx<float>*, const Cx<float>*, const int*, const Cx<float>*, Cx<float>*,
                                       const int*, int, size_t, int, double, hipStream_t);
template hipError_t launch_vmul<double>(const Cx<double>*, const Cx<double>*, const int*, const Cx<double>*,
                                        Cx<double>*, const int*, int, size_t, int, double, hipStream_t);

}  // namespace lsop
