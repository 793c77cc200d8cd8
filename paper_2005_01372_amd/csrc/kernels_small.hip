// Small dense FP64 kernels of the preconditioner build: the truncation of an
// oversampled range-finder factorisation through an l x l SVD.
//
// Oversampling (not in the paper, which draws exactly r probes; Halko,
// Martinsson & Tropp 2011, Section 5): with l = k + p probes, Alg. 2 gives
// G0 V ~= Q W~^H with Q and W~ of l columns.  A thin QR W~ = Q2 R2 turns this
// into Q (R2^H) Q2^H, and the best rank-k approximation of the l x l core
// R2^H = U_b S V_b^H gives U = Q U_b(:, :k) S_k and W = Q2 V_b(:, :k).
#include <cmath>

#include "internal.hpp"

namespace lsop {

// One-sided (Hestenes) Jacobi SVD of B = R2^H in one workgroup, FP64.
// Columns of B are the conjugated rows of R2 (row-major l x l), so the working
// copy Bc[j][i] = B[i][j] is read row by row.  Each sweep visits every column
// pair once in round-robin order (l / 2 disjoint pairs per round, one thread
// per pair): the pair's 2 x 2 Gram matrix [[a, g], [conj(g), b]] is
// diagonalised by a unitary rotation (the phase of g, then a real Jacobi
// rotation), applied to the two columns of B and of V.  Sweeps stop when no
// pair has |g| > tol sqrt(a b).  Then B V = U_b S: the rotated columns sorted
// by norm give M[a][c] = (B V)[a][col(c)] (c < k: U_b S_k) and
// Mp[a][c] = V[a][col(c)] (V_b(:, :k)); kept = number of those with a
// non-zero norm.
__global__ __launch_bounds__(256) void k_svd_jacobi(const Cx<double>* __restrict__ R2, int l, int k,
                                                    Cx<double>* __restrict__ Bc, Cx<double>* __restrict__ Vc,
                                                    Cx<double>* __restrict__ M, Cx<double>* __restrict__ Mp,
                                                    int* __restrict__ kept, double tol) {
  __shared__ int rot;
  __shared__ double sig[256];
  const int m = l + (l & 1);
  for (int idx = threadIdx.x; idx < l * l; idx += blockDim.x) {
    const int j = idx / l, i = idx % l;
    const Cx<double> v = R2[idx];
    Bc[idx] = Cx<double>{v.re, -v.im};
    Vc[idx] = Cx<double>{i == j ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (threadIdx.x == 0) rot = 0;
    __syncthreads();
    for (int r = 0; r < m - 1; ++r) {
      const int t = threadIdx.x;
      if (t < m / 2) {
        const int p = (r + t) % (m - 1);
        const int q = t ? (r - t + m - 1) % (m - 1) : m - 1;
        if (p < l && q < l) {
          Cx<double>* x = Bc + (size_t)p * l;
          Cx<double>* y = Bc + (size_t)q * l;
          double a = 0.0, b = 0.0, gre = 0.0, gim = 0.0;
          for (int i = 0; i < l; ++i) {
            const Cx<double> xi = x[i], yi = y[i];
            a += xi.re * xi.re + xi.im * xi.im;
            b += yi.re * yi.re + yi.im * yi.im;
            gre += xi.re * yi.re + xi.im * yi.im;  // conj(x) y
            gim += xi.re * yi.im - xi.im * yi.re;
          }
          const double ag = sqrt(gre * gre + gim * gim);
          if (ag > 0.0 && ag > tol * sqrt(a * b)) {
            rot = 1;
            // e^{-i phi} with g = |g| e^{i phi}; then the real rotation of [[a, |g|], [|g|, b]]
            const double er = gre / ag, ei = -gim / ag;
            const double zeta = (b - a) / (2.0 * ag);
            const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
            for (int w = 0; w < 2; ++w) {
              Cx<double>* X = (w ? Vc : Bc) + (size_t)p * l;
              Cx<double>* Y = (w ? Vc : Bc) + (size_t)q * l;
              for (int i = 0; i < l; ++i) {
                const Cx<double> xx = X[i];
                const Cx<double> yv = Y[i];
                const Cx<double> yy{yv.re * er - yv.im * ei, yv.re * ei + yv.im * er};
                X[i] = Cx<double>{c * xx.re - s * yy.re, c * xx.im - s * yy.im};
                Y[i] = Cx<double>{s * xx.re + c * yy.re, s * xx.im + c * yy.im};
              }
            }
          }
        }
      }
      __syncthreads();
    }
    const int any = rot;
    __syncthreads();
    if (!any) break;
  }
  for (int j = threadIdx.x; j < l; j += blockDim.x) {
    double s2 = 0.0;
    for (int i = 0; i < l; ++i) {
      const Cx<double> v = Bc[(size_t)j * l + i];
      s2 += v.re * v.re + v.im * v.im;
    }
    sig[j] = sqrt(s2);
  }
  __syncthreads();
  double smax = 0.0;
  for (int j = 0; j < l; ++j) smax = fmax(smax, sig[j]);
  for (int j = threadIdx.x; j < l; j += blockDim.x) {
    int rank = 0;
    for (int i = 0; i < l; ++i) rank += (sig[i] > sig[j] || (sig[i] == sig[j] && i < j)) ? 1 : 0;
    if (rank < k) {
      for (int a = 0; a < l; ++a) {
        M[(size_t)a * k + rank] = Bc[(size_t)j * l + a];
        Mp[(size_t)a * k + rank] = Vc[(size_t)j * l + a];
      }
      if (sig[j] > 1e-14 * smax) atomicAdd(kept, 1);
    }
  }
}

hipError_t launch_svd_trunc(const Cx<double>* R2, int l, int k, Cx<double>* Bc, Cx<double>* Vc, Cx<double>* M,
                            Cx<double>* Mp, int* kept, hipStream_t s) {
  if (l < 1 || l > 256 || k < 1 || k > l) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_svd_jacobi, dim3(1), dim3(256), 0, s, R2, l, k, Bc, Vc, M, Mp, kept, 1e-15);
  return hipGetLastError();
}

}  // namespace lsop
