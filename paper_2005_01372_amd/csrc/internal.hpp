// Internal declarations shared by the C ABI and the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/lsop.h"
#include "cx.hpp"

namespace lsop {

// Supported FFT lengths (each padded axis is 2 L >= 2 N).
int fft_length_for(int n);
// Also the short x-lengths 2, 4, 8, 16 of narrow sub-domains.
int fft_length_sub(int n);

// Error reporting (per thread).
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);
// Every device allocation of the library goes through these (counted for lsop_alloc_count).
hipError_t lib_malloc(void** p, size_t nbytes);
hipError_t lib_malloc_async(void** p, size_t nbytes, hipStream_t s);

#define LSOP_HIP(...)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (__VA_ARGS__);                                                          \
    if (e_ != hipSuccess)                                                                   \
      return ::lsop::fail(LSOP_EHIP, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ----------------------------------------------------------------- FFT path
// All launchers take the stream and return hipError_t of the launch.
// T = float or double.

// One vector of a grouped launch over several operators of the same shape.
template <typename T>
struct Slot {
  const Cx<T>* x;    // input vector (nx * nz)
  Cx<T>* y;          // output vector
  const Cx<T>* rhs;  // right-hand side of the residual epilogue, or NULL
  const T* chi;      // the operator's contrast
  const Cx<T>* gs;   // the operator's spectrum
  double* rnorm;     // |y|^2 accumulator (residual epilogue), or NULL
};
// Sub-domain batches (nodes > 1): each stored vector holds `nodes` strips of nx
// rows, transformed independently (slot = vector * nodes + node, chi sliced per
// strip); rows outside [lo, hi) of a strip are read as zero (hi < 0: nx).
// Grouped batches (tab != NULL, nodes = 1, no vidx): slot s takes its operands from tab[s].
// trows: rows per slot of tmp (default nx): a slot's rows i < nx are written to tmp rows slot * trows + i (the
// 3D operator stores each x-plane's ny rows in a plane of py rows).
// rm: which strip rows the pass visits.  Item i of a slot (0 <= i < rm.ns, default nx) is strip row
// rm.xa + rm.xs * i (xs = +1 or -1) and row i of the slot's part of tmp; the default visits every row in order.
// Sub-domain convolutions between the two halves of a node use it to move one half only, reflected or not.
struct RowMap {
  int ns = -1, xa = 0, xs = 1;
};
template <typename T>
hipError_t launch_rows_fwd(int L, const Cx<T>* x, const T* chi, Cx<T>* tmp, const int* vidx, int nx, int nz,
                           int nslots, bool mulchi, const Cx<T>* tw2, hipStream_t s, int nodes = 1, int lo = 0,
                           int hi = -1, const Slot<T>* tab = nullptr, int trows = -1, RowMap rm = RowMap());
// tile: columns per workgroup (0 = widest that fits; narrower tiles allow more workgroups per CU)
// *used (optional) receives the tile width launched
template <typename T>
hipError_t launch_cols(int L, Cx<T>* tmp, const Cx<T>* gs, int nx, int pz, int nslots, bool adj, const Cx<T>* tw2,
                       hipStream_t s, int tile = 0, int* used = nullptr, const Slot<T>* tab = nullptr);
// epi: 0 y = x - c, 1 y = c, 2 y = x - chi c, 3 y = chi c; rhs != NULL: y -= rhs and rnorm[slot] += |y|^2
// Sub-domain batches as in pass 1; rows outside [lo, hi) of a strip are not written.  The residual norm of
// a slot accumulates into rnorm[slot / nodes] (one norm per stored vector).  rm as in pass 1.
template <typename T>
hipError_t launch_rows_inv(int L, const Cx<T>* tmp, const Cx<T>* x, const T* chi, const Cx<T>* rhs, Cx<T>* y,
                           double* rnorm, const int* vidx, int nx, int nz, int nslots, int epi, const Cx<T>* tw2,
                           hipStream_t s, int nodes = 1, int lo = 0, int hi = -1, const Slot<T>* tab = nullptr,
                           int trows = -1, RowMap rm = RowMap());
// spectrum of the circulant-extended kernel table (FP64), written as gs[2][pz][lx] in T.
// circ = false: the x-lags are embedded symmetrically in the period 2 lx (lag min(p, 2 lx - p)), the table of
// a linear convolution.  circ = true: period 2 lx holds lag p itself at position p (a circular convolution whose
// inputs and outputs lie in opposite halves of the period, so that only lags 1 .. 2 lx - 1 occur), and the odd
// frequency half is negated, so that the even/odd recombination of the column pass returns the second half of
// the period.
hipError_t launch_spectrum(int lx, int lz, const Cx<double>* ktab, int nx, int nz, Cx<double>* s1t,
                           Cx<double>* gs64, Cx<float>* gs32, const Cx<double>* tw2x, const Cx<double>* tw2z,
                           hipStream_t s, bool circ = false);
// 3D operator: forward-only (dir 0) / inverse-only (dir 1) column transforms over slots of [rows_slot][pz]
// (dir 0: rows < nrow in, 2L rows out in split order; dir 1: 2L rows in, rows < nrow out); the 3D lag table
// (K = c1 e^{i k0 r} / r, K(0) = self); its spectrum gs[2][py pz][lx] (u: nx ny nz, F: px py pz complex doubles
// of workspace); incident fields of sources src[3 k + {0, 1, 2}] = (i, j, l).
template <typename T>
hipError_t launch_cols_half(int dir, int L, Cx<T>* tmp, int rows_slot, int nrow, int pz, int nslots,
                            const Cx<T>* tw2, hipStream_t s);
hipError_t launch_table3(Cx<double>* ktab, int nx, int ny, int nz, double k0, double h, double c1, Cx<double> self,
                         hipStream_t s);
hipError_t launch_spectrum3(int lx, int ly, int lz, const Cx<double>* ktab, int nx, int ny, int nz, Cx<double>* u,
                            Cx<double>* F, Cx<double>* gs64, Cx<float>* gs32, const Cx<double>* tw2x,
                            const Cx<double>* tw2y, const Cx<double>* tw2z, hipStream_t s);
template <typename T>
hipError_t launch_incident3(const Cx<double>* ktab, const int* src, const Cx<double>* amp, Cx<T>* out, int nx,
                            int ny, int nz, int nsrc, double inv_dv, hipStream_t s);
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
// y[vi] = a*x[vi] + b*y[vi] (real a, b) over nvec vectors of length n, indexed through vidx; a term whose
// coefficient is 0 is not read
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
// probes k0 .. k0 + nvec - 1 of the Philox stream with key `seed`
template <typename T>
hipError_t launch_philox_normal(Cx<T>* out, int nvec, size_t n, uint64_t seed, hipStream_t s, int k0 = 0);

// C[a][b] = sum_k conj(A[a][k]) B[vb][k], FP64 result (na x nb, ldc = nb).  B vectors through vidx.
// part: workspace for split-K partials (ksplit * na * nb complex doubles).
template <typename T>
hipError_t launch_gemm_ah_b(const Cx<T>* A, int na, const Cx<T>* B, const int* vidx, int nb, size_t n,
                            Cx<double>* C, Cx<double>* part, int ksplit, hipStream_t s);
// The split of C = A^H B: `nseg` segments of `seg` elements, each cut into ksub chunks of `chunk`.
struct GemmPlan {
  size_t seg = 0, chunk = 0;
  int nseg = 1, ksub = 1;
};
GemmPlan gemm_ah_b_plan(size_t n, size_t seg, int ksub);
// the two launches of the segmented product: partials (nseg * ksub * na * nb) and their reduction
// out32 != NULL (plans of one chunk per segment only): the products are written rounded to FP32 there, in
// the layout of the reduced result, instead of the partials.
template <typename T>
hipError_t launch_gemm_ah_b_part(const Cx<T>* A, int na, const Cx<T>* B, const int* vidx, int nb, size_t n,
                                 const GemmPlan& p, Cx<double>* part, hipStream_t s, Cx<float>* out32 = nullptr);
// C32 != NULL: the sums are written rounded to FP32 there (C unused).
hipError_t launch_reduce_parts(const Cx<double>* part, const GemmPlan& p, size_t count, Cx<double>* C, double alpha,
                               hipStream_t s, Cx<float>* C32 = nullptr);
// Segmented form: one na x nb result per segment of `seg` elements of k, at
// C + sg * na * nb; each segment split into ksub partial chunks (part holds
// nseg * ksub * na * nb complex doubles).
template <typename T>
hipError_t launch_gemm_ah_b_seg(const Cx<T>* A, int na, const Cx<T>* B, const int* vidx, int nb, size_t n, size_t seg,
                                Cx<double>* C, Cx<double>* part, int ksub, hipStream_t s, double alpha = 1.0);
// Y[vy(b)][k] = X1[vy(b)][k] + beta * X2[vy(b)][k] + sum_a A[a][k] M[a][b]   (M FP64, na x nb)
// X1 / X2 may be NULL (treated as 0).
template <typename T>
hipError_t launch_gemm_update(const Cx<T>* A, int na, const Cx<double>* M, int nb, const Cx<T>* X1,
                              const Cx<T>* X2, double beta, Cx<T>* Y, const int* vidx, size_t n, hipStream_t s);
// Segmented form: element k uses M + (k / seg) * mstride; seg must be a multiple of 64.  M in MT: FP64, or
// FP32 for complex-float T (coefficients that are FP32 values already, as the cores' FP32 products are).
// Y may be A itself (in place) when na == nb <= 64.
template <typename T, typename MT>
hipError_t launch_gemm_update_seg(const Cx<T>* A, int na, const Cx<MT>* M, size_t mstride, int nb,
                                  const Cx<T>* X1, const Cx<T>* X2, double beta, Cx<T>* Y, const int* vidx, size_t n,
                                  size_t seg, hipStream_t s);
// small FP64 dense kernels (one workgroup per batch entry, entries na * na apart); gram_orth: na <= 64
// gnorm (optional): the drop test's reference squared column norms, na per batch entry (default: G's own diagonal)
hipError_t launch_gram_orth(const Cx<double>* G, Cx<double>* X, int na, double drop_tol, int* kept, hipStream_t s,
                            int batch = 1, const double* gnorm = nullptr);
// out[sg * na + c] = squared 2-norm of row c of Y (na rows of n) over segment sg (nseg segments of seg elements)
template <typename T>
hipError_t launch_seg_colnorm2(const Cx<T>* Y, int na, size_t n, size_t seg, int nseg, double* out, hipStream_t s);
// Z_b = (I - M_b)^{-1} (plain = false) or M_b^{-1} (plain = true); M_b = M + b * sm (leading dimension ldm),
// Z_b likewise (may alias M_b); work: batch * 2 na^2 complex doubles when na > 64; singular[b] set to 1 on
// failure (the caller clears it).
hipError_t launch_lu_inverse(const Cx<double>* M, size_t ldm, size_t sm, Cx<double>* Z, size_t ldz, size_t sz,
                             Cx<double>* work, int na, bool plain, int* singular, int batch, hipStream_t s);
hipError_t launch_lu_inverse_i_minus(const Cx<double>* M, Cx<double>* Z, Cx<double>* work, int na, int* singular,
                                     hipStream_t s);
// C_b = alpha * A_b (na x na) * B_b (na x nb)
hipError_t launch_small_gemm(const Cx<double>* A, const Cx<double>* B, Cx<double>* C, int na, int nb, double alpha,
                             hipStream_t s, int batch = 1);
// FP32 Gauss-Jordan inverses of batch blocks of na <= 64 (as launch_lu_inverse, plain form)
hipError_t launch_lu_inverse_small_f32(const Cx<float>* M, size_t ldm, size_t sm, Cx<float>* Z, size_t ldz, size_t sz,
                                      int na, bool plain, int* singular, int batch, hipStream_t s);
// Truncation of an oversampled factorisation: one-sided Jacobi SVD of R2^H (R2 row-major l x l, FP64) in one
// workgroup; M = (U_b S)(:, :k) and Mp = V_b(:, :k), both row-major l x k; Bc, Vc: l * l work each; *kept
// (cleared by the caller) receives the number of non-zero singular values among the k kept.  l <= 256.
hipError_t launch_svd_trunc(const Cx<double>* R2, int l, int k, Cx<double>* Bc, Cx<double>* Vc, Cx<double>* M,
                            Cx<double>* Mp, int* kept, hipStream_t s);
// Krylov kernels (restarted GMRES), basis stored [i][vector][n] with block stride bstride, vectors through
// vidx[a], a < na.  mdot: h[a * hstride + i] (+)= sum_k conj(V[i][vs][k]) w[vs][k] for i < nb, through the
// partial sums part (na * nb * mdot_chunks(n) entries).  mcombine: out[vs] = beta out[vs] + alpha
// sum_i coef[a * cstride + i] V[i][vs].  scale_by_norm: y[vs] = sign x[vs] / sqrt(nrm2[a]) (0 where nrm2 = 0).
int mdot_chunks(size_t n);
template <typename T>
hipError_t launch_mdot(const Cx<T>* V, size_t bstride, int nb, const Cx<T>* w, const int* vidx, int na, size_t n,
                       Cx<double>* part, Cx<double>* h, int hstride, bool accumulate, hipStream_t s);
template <typename T>
hipError_t launch_mcombine(const Cx<T>* V, size_t bstride, int nb, const Cx<double>* coef, int cstride, double alpha,
                           double beta, Cx<T>* out, const int* vidx, int na, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_scale_by_norm(const Cx<T>* x, Cx<T>* y, const double* nrm2, double sign, const int* vidx, int na,
                                size_t n, hipStream_t s);
// Convergent Born series: kernel table at complex wavenumber (complex kh = k h), the potential
// V_eps = chi - i eps r (absorbing-layer profile r, see lsop_set_problem_damped) in FP64 and FP32 (either may be
// NULL), and pointwise products with it (x through xidx, y through yidx, c compact): op 0 y = V x,
// 1 y = x - conj(V) c, 2 y = conj(V) c, 3 y = gamma x, 4 y = y - gamma x, gamma = i V scale (scale = 1 / eps).
hipError_t launch_table_c(Cx<double>* ktab, int nx, int nz, Cx<double> kh, Cx<double> cj1, Cx<double> self,
                          hipStream_t s);
hipError_t launch_damped_potential(const double* chi, int nx, int nz, double eps, int absorb, Cx<double>* v64,
                                   Cx<float>* v32, hipStream_t s);
template <typename T>
hipError_t launch_vmul(const Cx<T>* V, const Cx<T>* x, const int* xidx, const Cx<T>* c, Cx<T>* y, const int* yidx,
                       int nvec, size_t n, int op, double scale, hipStream_t s);
// HODLR: dense leaf blocks of I - G0 V (formed in FP64, stored as To), leaves leaf0 .. leaf0 + nleaf - 1 of nl cells
template <typename To>
hipError_t launch_leaf_form(const Cx<double>* ktab, const double* chi, Cx<To>* out, int nz, int nl, int leaf0,
                            int nleaf, hipStream_t s);
// out_b = transpose(in_b), FP32 (m x m each)
hipError_t launch_transpose_f32(const Cx<float>* in, Cx<float>* out, int m, int batch, hipStream_t s);
// out_b = transpose(in_b) converted to T (m x m each)
template <typename T>
hipError_t launch_transpose_convert(const Cx<double>* in, Cx<T>* out, int m, int batch, hipStream_t s);
// batched complex GEMM C_b = alpha A_b B_b + beta C_b (rows of A / C through mapa / mapc when given)
template <typename T>
hipError_t launch_bgemm(const Cx<T>* A, size_t lda, size_t sA, const Cx<T>* B, size_t ldb, size_t sB, Cx<T>* C,
                        size_t ldc, size_t sC, const int* mapa, const int* mapc, int M, int N, int K, double alpha,
                        double beta, int batch, hipStream_t s);
// r x r identity blocks (leading dimension ld, batch stride st)
hipError_t launch_set_identity(Cx<double>* out, size_t ld, size_t st, int r, int batch, hipStream_t s);
// dev[b] = max |P_b - I| entrywise
hipError_t launch_identity_deviation(const Cx<double>* P, size_t ld, size_t st, int r, int batch, double* dev,
                                     hipStream_t s);
// p[0 .. count) = 0 (fill kernel, graph-capturable)
hipError_t launch_zero_f64(double* p, size_t count, hipStream_t s);
// zero the output vectors (tab[s].y, n elements) of the slots with live[s] == 0
template <typename T>
hipError_t launch_mask_slots(const Slot<T>* tab, const int* live, int nslots, size_t n, hipStream_t s);
// y[yidx[v]] += a * x[v] for v < nvec (x compact)
template <typename T>
hipError_t launch_axpy_map(const Cx<T>* x, Cx<T>* y, const int* yidx, double a, int nvec, size_t n, hipStream_t s);

// Runs one kernel launch; while the library's profiler is on, brackets it with
// events on stream s and records the use label, the kernel function name and
// the launch's algorithmic bytes and flops.
hipError_t prof_launch(const char* name, const char* fn, double bytes, double flops, double items, hipStream_t s,
                       const std::function<hipError_t()>& launch);

// The operator's FFT intermediate per vector, and y = op(x) with a caller-chosen intermediate of `chunk`
// vectors (the passes of lsop_apply, chunk by chunk).
size_t apply_tmp_bytes_per_vec(const lsop_op* op);
int apply_into(lsop_op* op, int mode, const void* x, void* y, int nvec, void* tmp, int chunk, hipStream_t s);

}  // namespace lsop

// ------------------------------------------------------------------ handles
struct lsop_op {
  int nx = 0, nz = 0, lx = 0, lz = 0, dtype = 0, max_vec = 0;
  int ny = 1, ly = 0, dims = 2;  // 3D operators (lsop_create3d): ny cells along y, y FFT length ly
  int col_tile = 0;  // column-pass tile width (0 = widest that fits)
  bool ready = false;
  double h = 0, freq = 0, c0 = 0, k0 = 0;
  size_t n() const { return (size_t)nx * ny * nz; }
  int px() const { return 2 * lx; }
  int py() const { return dims == 3 ? 2 * ly : 1; }
  int pz() const { return 2 * lz; }
  bool has64() const { return dtype != LSOP_C64; }
  bool has32() const { return dtype != LSOP_C128; }
  // device state
  double* chi64 = nullptr;
  float* chi32 = nullptr;
  Cx<double>* ktab = nullptr;                   // [nx][nz]
  Cx<double>* gs64 = nullptr;                   // [2][pz][lx]
  Cx<float>* gs32 = nullptr;
  Cx<double>*tw2x64 = nullptr, *tw2z64 = nullptr, *tw2y64 = nullptr;  // w_{2L}^t, t < 2L
  Cx<float>*tw2x32 = nullptr, *tw2z32 = nullptr, *tw2y32 = nullptr;
  void* tmp = nullptr;                          // [max_vec][nx][py][pz] in the widest dtype (py = 1 in 2D)
  unsigned* flag = nullptr;
  int* dsrc = nullptr;                          // sources (2 * cap) + vidx scratch
  Cx<double>* damp = nullptr;
  int src_cap = 0;
  size_t bytes = 0;
  // growable scratch for solvers (or the caller's workspace, see lsop_attach_workspace)
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  bool ws_external = false;     // scratch is the caller's: never grown, reallocated or freed
  // convergent Born series (lsop_set_problem_damped): dissipative background and complex potential
  bool damped = false;
  double eps = 0.0;
  Cx<double>* v64 = nullptr;    // V_eps = chi - i eps r, [nx][nz]
  Cx<float>* v32 = nullptr;
  void* vtmp = nullptr;         // [max_vec][n] pointwise products around the convolution
  bool state_external = false;  // device state carved from the caller's buffer (lsop_create_in)
  std::vector<void*> owned;
};

// One level of the HODLR preconditioner (nodes of `width` grid columns).
struct hodlr_level {
  int width = 0, lx = 0;                  // node width and its x-FFT length
  bool half = false;                      // sampling convolves half-node to half-node at period width (lx = width / 2)
  void* V = nullptr;                      // [rank][n] packed right factors (per half-node)
  void* Wp = nullptr;                     // [rank][n] A_{l+1}^{-1} U, packed
  Cx<double>* kinv = nullptr;             // [nodes][2 rank][2 rank] (P K)^{-1}
  Cx<float>* kinv32 = nullptr;            // its FP32 copy (complex-FP32 preconditioners apply the cores in FP32)
  Cx<double>* gs64 = nullptr;             // sub-domain spectrum [2][pz][lx]
  Cx<float>* gs32 = nullptr;
  Cx<double>* tw64 = nullptr;             // x twiddles w_{2 lx}
  Cx<float>* tw32 = nullptr;
};

struct lsop_precond {
  lsop_op* op = nullptr;
  int kind = 0, rank = 0, q = 0, kept = 0;
  int q_from = 0;  // HODLR: power iterations on levels >= q_from only
  int probes = 0;          // probe vectors l = rank + oversample (LOWRANK)
  double alpha = 0.0;      // SCALAR: H = alpha I
  void* Q2 = nullptr;      // [probes][n] orthonormal basis of W~ (oversampled builds)
  Cx<double>* svdw = nullptr;  // R2, Bc, Vc (probes^2 each), M, Mp (probes * rank each)
  bool state_external = false;
  // HODLR (kind LSOP_PC_HODLR)
  int levels = 0, leaf_w = 0, nleaf = 0, leaf_chunk = 0;
  std::vector<hodlr_level> lev;
  void* dinv = nullptr;                   // [nleaf][nl][nl] transposed leaf inverses
  Cx<double>* lwork = nullptr;            // leaf workspace (leaf_chunk matrices + recursion temporaries, in the
                                          // leaves' precision; allocated in complex-double units)
  size_t lwork_elems = 0;
  void* hy = nullptr;                     // [tcap][n] apply / series temporary
  Cx<double>*hG = nullptr, *hX = nullptr;  // per-segment products [maxseg][rank][tcap]
  Cx<float>*hG32 = nullptr, *hX32 = nullptr;  // their FP32 copies around the FP32 core apply
  Cx<double>* hK = nullptr;               // node-core recursion temporaries and Gauss-Jordan work
  int* hflag = nullptr;                   // per-node / per-segment flags
  int maxseg = 0, ksub_cap = 0;
  uint64_t seed = 0;
  int dt = 0;              // storage dtype of U, W (LSOP_C64 or LSOP_C128)
  void* U = nullptr;       // [rank][n]
  void* W = nullptr;       // [rank][n]
  void* Y = nullptr;       // [rank][n] build workspace
  Cx<double>* Z = nullptr;     // [rank][rank]
  Cx<double>* small = nullptr; // gram / X / LU work / T buffers
  Cx<double>* part = nullptr;  // split-K partials
  size_t part_cap = 0;         // entries of part
  int* dflag = nullptr;
  int ksplit = 0;
  int tcap = 0;            // columns of the T buffers
  bool built = false;
  size_t bytes = 0;
  std::vector<void*> owned;
};

// A batch of operators of possibly different sizes, grouped by shape: every
// FFT pass is launched once per group over all vectors of its members.
struct lsop_batch {
  int count = 0, dtype = 0;
  std::vector<lsop_op*> ops;
  struct Group {
    int nx = 0, nz = 0, lx = 0, lz = 0, col_tile = 0;
    std::vector<int> members;
  };
  std::vector<Group> groups;
  std::vector<int> group_of;      // instance -> group
  void* tab = nullptr;            // slot tables of all groups (device)
  size_t tab_cap = 0;             // bytes
  void* tmp = nullptr;            // grouped intermediate (largest group)
  size_t tmp_cap = 0;
  void* work = nullptr;           // series: residual vectors, norms, live flags
  size_t work_cap = 0;
  std::vector<unsigned char> host_tab;
  size_t bytes = 0;
  // series: the per-instance preconditioner applies of an iteration run on these streams (forked from and
  // joined back into the series stream with ev: ev[0] the fork, ev[1 + k] the join of side[k])
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;
  int active_side = 0;            // side streams used by the current series
};
