// Internal declarations shared by the C ABI and the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lsop.h"
#include "cx.hpp"

namespace lsop {

// Supported FFT lengths (each padded axis is 2 L >= 2 N).
int fft_length_for(int n);

// Error reporting (per thread).
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);

#define LSOP_HIP(...)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (__VA_ARGS__);                                                          \
    if (e_ != hipSuccess)                                                                   \
      return ::lsop::fail(LSOP_EHIP, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ----------------------------------------------------------------- FFT path
// All launchers take the stream and return hipError_t of the launch.
// T = float or double.
template <typename T>
hipError_t launch_rows_fwd(int L, const Cx<T>* x, const T* chi, Cx<T>* tmp, const int* vidx, int nx, int nz,
                           int nslots, bool mulchi, const Cx<T>* tw2, hipStream_t s);
// tile: columns per workgroup (0 = widest that fits; narrower tiles allow more workgroups per CU)
template <typename T>
hipError_t launch_cols(int L, Cx<T>* tmp, const Cx<T>* gs, int nx, int pz, int nslots, bool adj, const Cx<T>* tw2,
                       hipStream_t s, int tile = 0);
// epi: 0 y = x - c, 1 y = c, 2 y = x - chi c, 3 y = chi c; rhs != NULL: y -= rhs and rnorm[slot] += |y|^2
template <typename T>
hipError_t launch_rows_inv(int L, const Cx<T>* tmp, const Cx<T>* x, const T* chi, const Cx<T>* rhs, Cx<T>* y,
                           double* rnorm, const int* vidx, int nx, int nz, int nslots, int epi, const Cx<T>* tw2,
                           hipStream_t s);
// spectrum of the circulant-extended kernel table (FP64), written as gs[2][pz][lx] in T
hipError_t launch_spectrum(int lx, int lz, const Cx<double>* ktab, int nx, int nz, Cx<double>* s1t,
                           Cx<double>* gs64, Cx<float>* gs32, const Cx<double>* tw2x, const Cx<double>* tw2z,
                           hipStream_t s);
hipError_t launch_contrast(const double* vel, double* chi64, float* chi32, int n, double w2, double inv_c02,
                           unsigned* bad, hipStream_t s);
hipError_t launch_table(Cx<double>* ktab, int nx, int nz, double k0h, Cx<double> cj1, Cx<double> self,
                        hipStream_t s);
template <typename T>
hipError_t launch_incident(const Cx<double>* ktab, const int* si, const int* sj, const Cx<double>* amp, Cx<T>* out,
                           int nx, int nz, int nsrc, double inv_dv, hipStream_t s);

// --------------------------------------------------------- vector / LA path
template <typename T>
hipError_t launch_norm2(const Cx<T>* x, double* out, const int* vidx, int nvec, size_t n, hipStream_t s);
template <typename To, typename Ti>
hipError_t launch_convert(const Cx<Ti>* x, Cx<To>* y, size_t count, hipStream_t s);
// y[vi] = a*x[vi] + b*y[vi] (real a, b) over nvec vectors of length n, indexed through vidx
template <typename T>
hipError_t launch_axpby(const Cx<T>* x, Cx<T>* y, double a, double b, const int* vidx, int nvec, size_t n,
                        hipStream_t s);
// y[vi] (FP64) += alpha * x[vi] (T); used by refinement
template <typename T>
hipError_t launch_accumulate(const Cx<T>* x, Cx<double>* y, double alpha, const int* vidx, int nvec, size_t n,
                             hipStream_t s);
// real FP64 probes [l][n] -> complex T
template <typename T>
hipError_t launch_real_to_complex(const double* in, Cx<T>* out, size_t count, hipStream_t s);
template <typename T>
hipError_t launch_philox_normal(Cx<T>* out, int nvec, size_t n, uint64_t seed, hipStream_t s);

// C[a][b] = sum_k conj(A[a][k]) B[vb][k], FP64 result (na x nb, ldc = nb).  B vectors through vidx.
// part: workspace for split-K partials (ksplit * na * nb complex doubles).
template <typename T>
hipError_t launch_gemm_ah_b(const Cx<T>* A, int na, const Cx<T>* B, const int* vidx, int nb, size_t n,
                            Cx<double>* C, Cx<double>* part, int ksplit, hipStream_t s);
// Y[vy(b)][k] = X1[vy(b)][k] + beta * X2[vy(b)][k] + sum_a A[a][k] M[a][b]   (M FP64, na x nb)
// X1 / X2 may be NULL (treated as 0).
template <typename T>
hipError_t launch_gemm_update(const Cx<T>* A, int na, const Cx<double>* M, int nb, const Cx<T>* X1,
                              const Cx<T>* X2, double beta, Cx<T>* Y, const int* vidx, size_t n, hipStream_t s);
// small FP64 dense kernels (one workgroup)
hipError_t launch_gram_orth(const Cx<double>* G, Cx<double>* X, int na, double drop_tol, int* kept,
                            hipStream_t s);
hipError_t launch_lu_inverse_i_minus(const Cx<double>* M, Cx<double>* Z, Cx<double>* work, int na, int* singular,
                                     hipStream_t s);
// C = alpha * A (na x na) * B (na x nb)
hipError_t launch_small_gemm(const Cx<double>* A, const Cx<double>* B, Cx<double>* C, int na, int nb, double alpha,
                             hipStream_t s);

}  // namespace lsop

// ------------------------------------------------------------------ handles
struct lsop_op {
  int nx = 0, nz = 0, lx = 0, lz = 0, dtype = 0, max_vec = 0;
  int col_tile = 0;  // column-pass tile width (0 = widest that fits)
  bool ready = false;
  double h = 0, freq = 0, c0 = 0, k0 = 0;
  size_t n() const { return (size_t)nx * nz; }
  int px() const { return 2 * lx; }
  int pz() const { return 2 * lz; }
  bool has64() const { return dtype != LSOP_C64; }
  bool has32() const { return dtype != LSOP_C128; }
  // device state
  double* chi64 = nullptr;
  float* chi32 = nullptr;
  Cx<double>* ktab = nullptr;                   // [nx][nz]
  Cx<double>* gs64 = nullptr;                   // [2][pz][lx]
  Cx<float>* gs32 = nullptr;
  Cx<double>*tw2x64 = nullptr, *tw2z64 = nullptr;  // w_{2L}^t, t < 2L
  Cx<float>*tw2x32 = nullptr, *tw2z32 = nullptr;
  void* tmp = nullptr;                          // [max_vec][nx][pz] in the widest dtype
  unsigned* flag = nullptr;
  int* dsrc = nullptr;                          // sources (2 * cap) + vidx scratch
  Cx<double>* damp = nullptr;
  int src_cap = 0;
  size_t bytes = 0;
  // growable scratch for solvers
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  std::vector<void*> owned;
};

struct lsop_precond {
  lsop_op* op = nullptr;
  int kind = 0, rank = 0, q = 0, kept = 0;
  uint64_t seed = 0;
  int dt = 0;              // storage dtype of U, W (LSOP_C64 or LSOP_C128)
  void* U = nullptr;       // [rank][n]
  void* W = nullptr;       // [rank][n]
  void* Y = nullptr;       // [rank][n] build workspace
  Cx<double>* Z = nullptr;     // [rank][rank]
  Cx<double>* small = nullptr; // gram / X / LU work / T buffers
  Cx<double>* part = nullptr;  // split-K partials
  int* dflag = nullptr;
  int ksplit = 0;
  int tcap = 0;            // columns of the T buffers
  bool built = false;
  size_t bytes = 0;
  std::vector<void*> owned;
};
