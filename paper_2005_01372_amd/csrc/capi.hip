// C ABI of liblsop.so: operator, preconditioner and series solver handles.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "bessel.hpp"
#include "bessel_complex.hpp"
#include "internal.hpp"

namespace lsop {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
int fail(int status, const std::string& msg) {
  g_err = msg;
  return status;
}

// Device allocations the library makes (diagnostic: caller-owned handles must not add any).
std::atomic<size_t> g_allocs{0};

hipError_t lib_malloc(void** p, size_t nbytes) {
  ++g_allocs;
  return hipMalloc(p, nbytes);
}

hipError_t lib_malloc_async(void** p, size_t nbytes, hipStream_t s) {
  ++g_allocs;
  return hipMallocAsync(p, nbytes, s);
}

namespace {

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------------ profiler
struct ProfRec {
  std::string name, fn;  // use label, kernel function
  hipEvent_t a, b;
  double bytes, flops, items;
};
bool g_prof = false;
std::vector<ProfRec> g_recs;
std::vector<hipEvent_t> g_pool;
std::mutex g_prof_mu;  // guards g_recs and g_pool: builds may run on several host threads

hipEvent_t ev_get() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Runs `launch` (one kernel launch, returning hipError_t); while profiling,
// brackets it with events on its stream and records the use label, the kernel
// function `fn` (read after the launch, so the launch may fill it in) and the
// launch's algorithmic bytes and flops.
template <typename F>
hipError_t prof(const char* name, const std::string& fn, double bytes, double flops, double items, hipStream_t s,
                F&& launch) {
  if (!g_prof) return launch();
  ProfRec r{name, "", nullptr, nullptr, bytes, flops, items};
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    r.a = ev_get();
    r.b = ev_get();
  }
  (void)hipEventRecord(r.a, s);
  hipError_t e = launch();
  (void)hipEventRecord(r.b, s);
  r.fn = fn;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_recs.push_back(r);
  return e;
}

template <typename T>
const char* tname();
template <>
const char* tname<float>() { return "float"; }
template <>
const char* tname<double>() { return "double"; }

std::string fn_name(const char* base, const char* t, int a = -1, int b = -1, int c = -1) {
  std::string f = std::string(base) + "<" + t;
  if (a >= 0) f += ", " + std::to_string(a);
  if (b >= 0) f += ", " + std::to_string(b);
  if (c >= 0) f += ", " + std::to_string(c);
  return f + ">";
}

// Real flops per complex multiply-add of a GEMM kernel: 6 for the complex FP32 kernels, which take Gauss's 3M
// form (three real products), 8 for the two-chain form.
double cmac_flops(bool three_m) { return three_m ? 6.0 : 8.0; }

// C = alpha A^H B (segmented) as its two profiled launches
// Chunks per segment for C = A^H B: the caller's ksub, raised for launches with few 64 x 64 output tiles until
// there are about 2048 workgroups (8 per CU), while chunks keep at least 1024 elements and the partials fit the
// part_cap entries of the workspace.
int ksub_fill(size_t seg, int nseg, int na, int nb, int ksub, size_t part_cap) {
  const size_t tiles = (size_t)((na + 63) / 64) * ((nb + 63) / 64) * nseg;
  const size_t want = (2048 + tiles - 1) / tiles;
  const size_t most = std::min<size_t>(std::max<size_t>(1, seg / 1024), part_cap / ((size_t)nseg * na * nb));
  return (int)std::max<size_t>(ksub, std::min(want, most));
}

// C32 != NULL: the products are written rounded to FP32 there instead of C.
template <typename T>
hipError_t p_ah_b(const char* name, const Cx<T>* A, int na, const Cx<T>* B, const int* vidx, int nb, size_t n,
                  size_t seg, Cx<double>* C, Cx<double>* part, int ksub, hipStream_t s, double alpha = 1.0,
                  size_t part_cap = 0, Cx<float>* C32 = nullptr) {
  if (na <= 0 || nb <= 0) return hipSuccess;
  {
    const size_t sg = (seg == 0 || seg > n) ? n : seg;
    ksub = ksub_fill(sg, (int)((n + sg - 1) / sg), na, nb, ksub, part_cap);
  }
  const GemmPlan p = gemm_ah_b_plan(n, seg, ksub);
  const double e = sizeof(Cx<T>), nab = (double)na * nb * sizeof(Cx<double>), parts = (double)p.nseg * p.ksub;
  // FP32 results from one chunk per segment: the products themselves, no reduction launch
  const bool direct = C32 && p.ksub == 1 && alpha == 1.0;
  hipError_t err = prof(name, fn_name(nb <= 16 ? "k_gemm_ah_b_narrow" : "k_gemm_ah_b_mfma", tname<T>()),
                        (double)(na + nb) * n * e + (direct ? 0.5 : 1.0) * parts * nab,
                        cmac_flops(sizeof(T) == 4) * na * nb * (double)n, nb,
                        s, [&] {
                          return launch_gemm_ah_b_part<T>(A, na, B, vidx, nb, n, p, part, s, direct ? C32 : nullptr);
                        });
  if (err != hipSuccess || direct) return err;
  return prof(name, "k_reduce_parts", (parts + (C32 ? 0.5 : 1.0) * p.nseg) * nab, 2.0 * parts * na * nb, nb, s,
              [&] { return launch_reduce_parts(part, p, (size_t)na * nb, C, alpha, s, C32); });
}

// Y = X1 + beta X2 + A M (segmented; M in MT), profiled
template <typename T, typename MT = double>
hipError_t p_update(const char* name, const Cx<T>* A, int na, const Cx<MT>* M, size_t mstride, int nb,
                    const Cx<T>* X1, const Cx<T>* X2, double beta, Cx<T>* Y, const int* vidx, size_t n, size_t seg,
                    hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  const double e = sizeof(Cx<T>);
  const double vecs = 1.0 + (X1 ? 1.0 : 0.0) + (X2 ? 1.0 : 0.0);
  const double nsegs = (seg == 0 || seg >= n) ? 1.0 : (double)((n + seg - 1) / seg);
  // the kernel launch_gemm_update_seg picks
  const int nbt = nb > 32 ? 4 : nb > 16 ? 2 : 1, ga = nb > 32 ? 4 : 8, wpe = nb > 32 ? (sizeof(T) == 4 ? 6 : 3) : 0;
  const std::string types = std::string(tname<T>()) + ", " + tname<MT>();
  const std::string kname = (sizeof(T) == 4 && nb > 32) ? fn_name("k_gemm_update_tile", tname<MT>())
                                                         : fn_name("k_gemm_update_mfma", types.c_str(), nbt, ga, wpe);
  return prof(name, kname,
              (double)na * n * e + vecs * nb * (double)n * e + nsegs * na * nb * sizeof(Cx<MT>),
              cmac_flops(sizeof(T) == 4 && nb > 32) * na * nb * (double)n, nb, s,
              [&] { return launch_gemm_update_seg<T, MT>(A, na, M, mstride, nb, X1, X2, beta, Y, vidx, n, seg, s); });
}

// batched C = alpha A B + beta C, profiled
template <typename T>
hipError_t p_bgemm(const char* name, const Cx<T>* A, size_t lda, size_t sA, const Cx<T>* B, size_t ldb, size_t sB,
                   Cx<T>* C, size_t ldc, size_t sC, const int* mapa, const int* mapc, int M, int N, int K,
                   double alpha, double beta, int batch, hipStream_t s) {
  const double e = sizeof(Cx<T>);
  const double bytes = (double)batch * ((double)M * K + (double)K * N + (double)M * N * (beta != 0.0 ? 2.0 : 1.0)) * e;
  return prof(name, fn_name("k_bgemm_mfma", tname<T>()), bytes, cmac_flops(sizeof(T) == 4) * M * N * (double)K * batch,
              batch, s, [&] {
    return launch_bgemm<T>(A, lda, sA, B, ldb, sB, C, ldc, sC, mapa, mapc, M, N, K, alpha, beta, batch, s);
  });
}

double fft_flops(int L) { return 5.0 * L * std::log2((double)L); }

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Where a handle's device state comes from: the library (one hipMalloc per buffer, recorded in `owned`), the
// caller's buffer (base / cap: buffers carved at 256-byte aligned offsets), or nowhere (count_only: the size
// query walks the same plan and only adds up the aligned sizes).  `bytes` is the running total.
struct Alloc {
  std::vector<void*>* owned = nullptr;
  size_t* bytes = nullptr;
  char* base = nullptr;
  size_t cap = 0;
  bool count_only = false;
};

template <typename P>
int dev_alloc(Alloc& a, P** out, size_t nbytes) {
  *out = nullptr;
  nbytes = align_up(nbytes == 0 ? 16 : nbytes);
  if (a.count_only) {
    *a.bytes += nbytes;
    return LSOP_OK;
  }
  if (a.base) {
    if (*a.bytes + nbytes > a.cap)
      return fail(LSOP_ENOMEM, "caller's state buffer of " + std::to_string(a.cap) + " bytes is too small");
    *out = reinterpret_cast<P*>(a.base + *a.bytes);
    *a.bytes += nbytes;
    return LSOP_OK;
  }
  void* p = nullptr;
  if (lib_malloc(&p, nbytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LSOP_ENOMEM, "hipMalloc of " + std::to_string(nbytes) + " bytes failed");
  }
  a.owned->push_back(p);
  *a.bytes += nbytes;
  *out = reinterpret_cast<P*>(p);
  return LSOP_OK;
}

void free_all(std::vector<void*>& owned) {
  for (void* p : owned) (void)hipFree(p);
  owned.clear();
}

// w_{2L}^t = exp(-2 pi i t / (2L)) for t < 2L, evaluated in long double
std::vector<Cx<double>> twiddles(int L) {
  std::vector<Cx<double>> w(2 * L);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int t = 0; t < 2 * L; ++t) {
    const long double a = pi * (long double)t / (long double)L;
    w[t] = Cx<double>{(double)cosl(a), (double)(-sinl(a))};
  }
  return w;
}

// The operator's workspace of at least `need` bytes: the caller's attached workspace (never grown: too small is
// ENOMEM, reported before the call launches anything that depends on it) or a library buffer grown on demand.
int grow_scratch(lsop_op* op, size_t need) {
  if (need <= op->scratch_bytes) return LSOP_OK;
  if (op->ws_external)
    return fail(LSOP_ENOMEM, "the attached workspace of " + std::to_string(op->scratch_bytes) +
                                 " bytes is smaller than the " + std::to_string(need) + " bytes this call needs");
  if (op->scratch) {
    LSOP_HIP(hipDeviceSynchronize());
    (void)hipFree(op->scratch);
    op->scratch = nullptr;
    op->scratch_bytes = 0;
  }
  if (lib_malloc(&op->scratch, need) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LSOP_ENOMEM, "scratch allocation of " + std::to_string(need) + " bytes failed");
  }
  op->scratch_bytes = need;
  return LSOP_OK;
}

template <typename T>
struct Dt;
template <>
struct Dt<float> {
  static const float* chi(const lsop_op* op) { return op->chi32; }
  static const Cx<float>* gs(const lsop_op* op) { return op->gs32; }
  static const Cx<float>* twx(const lsop_op* op) { return op->tw2x32; }
  static const Cx<float>* twz(const lsop_op* op) { return op->tw2z32; }
  static const Cx<float>* twy(const lsop_op* op) { return op->tw2y32; }
};
template <>
struct Dt<double> {
  static const double* chi(const lsop_op* op) { return op->chi64; }
  static const Cx<double>* gs(const lsop_op* op) { return op->gs64; }
  static const Cx<double>* twx(const lsop_op* op) { return op->tw2x64; }
  static const Cx<double>* twz(const lsop_op* op) { return op->tw2z64; }
  static const Cx<double>* twy(const lsop_op* op) { return op->tw2y64; }
};

// y = op(x) (mode), or r = A x - rhs with norms when rhs != NULL.  Vectors are
// addressed through vidx (device, nvec entries) when given, else 0..nvec-1.
// tmp_in / chunk: an intermediate other than the operator's own, holding `chunk` vectors (default: op->tmp,
// max_vec vectors).
template <typename T>
int apply_impl(lsop_op* op, int mode, const Cx<T>* x, Cx<T>* y, const Cx<T>* rhs, double* rnorm, const int* vidx,
               int nvec, hipStream_t s, void* tmp_in = nullptr, int chunk = 0) {
  const size_t n = op->n();
  Cx<T>* tmp = reinterpret_cast<Cx<T>*>(tmp_in ? tmp_in : op->tmp);
  int step = chunk > 0 ? chunk : op->max_vec;
  const bool mulchi = (mode == LSOP_MODE_A || mode == LSOP_MODE_G0V);
  const bool adj = !mulchi;
  // dissipative background (convergent Born series): the complex potential multiplies outside the FFT passes,
  // through the operator's [max_vec][n] temporary
  const bool damped = op->damped;
  Cx<T>* vt = reinterpret_cast<Cx<T>*>(op->vtmp);
  const Cx<T>* Vp = damped ? reinterpret_cast<const Cx<T>*>(std::is_same<T, float>::value ? (const void*)op->v32
                                                                                            : (const void*)op->v64)
                           : nullptr;
  if (damped) step = std::min(step, op->max_vec);
  for (int c = 0; c < nvec; c += step) {
    const int m = std::min(step, nvec - c);
    const int* vc = vidx ? vidx + c : nullptr;
    const size_t off = vidx ? 0 : (size_t)c * n;
    double* rn = rnorm ? rnorm + c : nullptr;
    // algorithmic bytes: compulsory reads + writes of each pass (see the kernel file header)
    const double e = sizeof(Cx<T>), t = sizeof(T), nn = (double)n;
    const double np = (double)op->nx * op->pz();
    const double frow = 2.0 * fft_flops(op->lz) + 6.0 * op->lz;
    const double fcols = 4.0 * fft_flops(op->lx) + 18.0 * op->lx;
    const bool xin = (mode == LSOP_MODE_A || mode == LSOP_MODE_AH);
    const bool chi_out = (mode == LSOP_MODE_AH || mode == LSOP_MODE_VHG0H);
    if (op->dims == 3) {
      // 3D: z rows (x-plane i's ny rows stored in a plane of py rows), y columns forward per x-plane, x columns
      // with the spectrum (k_cols over the py pz columns), y columns inverse, z rows inverse with the epilogue
      const int py = op->py(), pz = op->pz(), planes = m * op->nx;
      const double np3 = (double)op->nx * py * pz;
      LSOP_HIP(prof("lsop3_rows_fwd", fn_name("k_rows_fwd", tname<T>(), op->lz),
                    m * (nn * e + np3 * e / 2) + (mulchi ? nn * t : 0.0), (double)planes * op->ny * frow, m, s, [&] {
                      return launch_rows_fwd<T>(op->lz, x + off, Dt<T>::chi(op), tmp, vc, op->ny, op->nz, planes,
                                                mulchi, Dt<T>::twz(op), s, op->nx, 0, op->ny, nullptr, py);
                    }));
      LSOP_HIP(prof("lsop3_cols_y", "k_cols_half", m * (np3 * e / 2 + np3 * e), (double)planes * pz *
                    2.0 * fft_flops(op->ly), m, s, [&] {
                      return launch_cols_half<T>(0, op->ly, tmp, py, op->ny, pz, planes, Dt<T>::twy(op), s);
                    }));
      LSOP_HIP(prof("lsop3_cols_x", fn_name("k_cols", tname<T>(), op->lx), m * 2.0 * np3 * e + np3 * e,
                    (double)m * py * pz * fcols, m, s, [&] {
                      return launch_cols<T>(op->lx, tmp, Dt<T>::gs(op), op->nx, py * pz, m, adj, Dt<T>::twx(op), s,
                                            op->col_tile);
                    }));
      LSOP_HIP(prof("lsop3_cols_y", "k_cols_half", m * (np3 * e + np3 * e / 2), (double)planes * pz *
                    2.0 * fft_flops(op->ly), m, s, [&] {
                      return launch_cols_half<T>(1, op->ly, tmp, py, op->ny, pz, planes, Dt<T>::twy(op), s);
                    }));
      LSOP_HIP(prof("lsop3_rows_inv", fn_name("k_rows_inv", tname<T>(), op->lz),
                    m * (np3 * e / 2 + nn * e + (xin ? nn * e : 0.0) + (rhs ? nn * e : 0.0)) +
                        (chi_out ? nn * t : 0.0),
                    (double)planes * op->ny * frow, m, s, [&] {
                      return launch_rows_inv<T>(op->lz, tmp, x + off, Dt<T>::chi(op), rhs ? rhs + off : nullptr,
                                                y + off, rn, vc, op->ny, op->nz, planes, mode, Dt<T>::twz(op), s,
                                                op->nx, 0, op->ny, nullptr, py);
                    }));
      continue;
    }
    if (damped) {
      // u = V x (forward modes) into the temporary; the passes then convolve without the real contrast
      const Cx<T>* xin1 = x + off;
      const int* vin1 = vc;
      if (mulchi) {
        LSOP_HIP(prof("damped_vmul", "k_vmul", 3.0 * m * n * sizeof(Cx<T>), 6.0 * m * n, m, s, [&] {
          return launch_vmul<T>(Vp, x + off, vc, nullptr, vt, nullptr, m, n, 0, 0.0, s);
        }));
        xin1 = vt;
        vin1 = nullptr;
      }
      LSOP_HIP(launch_rows_fwd<T>(op->lz, xin1, Dt<T>::chi(op), tmp, vin1, op->nx, op->nz, m, false, Dt<T>::twz(op),
                                  s));
      LSOP_HIP(launch_cols<T>(op->lx, tmp, Dt<T>::gs(op), op->nx, op->pz(), m, adj, Dt<T>::twx(op), s, op->col_tile));
      if (mulchi) {
        LSOP_HIP(launch_rows_inv<T>(op->lz, tmp, x + off, Dt<T>::chi(op), rhs ? rhs + off : nullptr, y + off, rn, vc,
                                    op->nx, op->nz, m, mode == LSOP_MODE_A ? 0 : 1, Dt<T>::twz(op), s));
      } else {
        // c = G^H x into the temporary, then y = x - conj(V) c (AH) or conj(V) c (VHG0H)
        LSOP_HIP(launch_rows_inv<T>(op->lz, tmp, nullptr, Dt<T>::chi(op), nullptr, vt, nullptr, nullptr, op->nx,
                                    op->nz, m, 1, Dt<T>::twz(op), s));
        LSOP_HIP(prof("damped_vmul", "k_vmul", 3.0 * m * n * sizeof(Cx<T>), 6.0 * m * n, m, s, [&] {
          return launch_vmul<T>(Vp, x + off, vc, vt, y + off, vc, m, n, mode == LSOP_MODE_AH ? 1 : 2, 0.0, s);
        }));
      }
      continue;
    }
    std::string fcol;
    LSOP_HIP(prof("lsop_rows_fwd", fn_name("k_rows_fwd", tname<T>(), op->lz), m * (nn * e + np * e) + (mulchi ? nn * t : 0.0),
                  (double)m * op->nx * frow, m, s, [&] {
                    return launch_rows_fwd<T>(op->lz, x + off, Dt<T>::chi(op), tmp, vc, op->nx, op->nz, m, mulchi,
                                              Dt<T>::twz(op), s);
                  }));
    LSOP_HIP(prof("lsop_cols", fcol, m * 2.0 * np * e + 2.0 * op->pz() * op->lx * e, (double)m * op->pz() * fcols, m, s,
                  [&] {
                    int used = 0;
                    hipError_t er = launch_cols<T>(op->lx, tmp, Dt<T>::gs(op), op->nx, op->pz(), m, adj, Dt<T>::twx(op),
                                                   s, op->col_tile, &used);
                    fcol = fn_name("k_cols", tname<T>(), op->lx, used);
                    return er;
                  }));
    LSOP_HIP(prof("lsop_rows_inv", fn_name("k_rows_inv", tname<T>(), op->lz),
                  m * (np * e + nn * e + (xin ? nn * e : 0.0) + (rhs ? nn * e : 0.0)) + (chi_out ? nn * t : 0.0),
                  (double)m * op->nx * frow, m, s, [&] {
                    return launch_rows_inv<T>(op->lz, tmp, x + off, Dt<T>::chi(op), rhs ? rhs + off : nullptr,
                                              y + off, rn, vc, op->nx, op->nz, m, mode, Dt<T>::twz(op), s);
                  }));
  }
  return LSOP_OK;
}

template <typename T>
hipError_t p_gemm_ah_b(const Cx<T>* A, int na, const Cx<T>* B, const int* vidx, int nb, size_t n, Cx<double>* C,
                       Cx<double>* part, int ksplit, hipStream_t s, size_t part_cap = 0) {
  return p_ah_b<T>("lsop_gemm_ah_b", A, na, B, vidx, nb, n, n, C, part, ksplit, s, 1.0, part_cap);
}

template <typename T>
hipError_t p_gemm_update(const Cx<T>* A, int na, const Cx<double>* M, int nb, const Cx<T>* X1, const Cx<T>* X2,
                         double beta, Cx<T>* Y, const int* vidx, size_t n, hipStream_t s) {
  return p_update<T>("lsop_gemm_update", A, na, M, 0, nb, X1, X2, beta, Y, vidx, n, n, s);
}

// Times the column pass for each tile width on the operator's shape (m vectors
// of whatever the intermediate buffer holds) and keeps the fastest.
template <typename T>
int autotune_cols(lsop_op* op, int m, hipStream_t s) {
  Cx<T>* tmp = reinterpret_cast<Cx<T>*>(op->tmp);
  hipEvent_t a, b;
  LSOP_HIP(hipEventCreate(&a));
  LSOP_HIP(hipEventCreate(&b));
  float best = 1e30f;
  int best_tile = 0;
  for (int tile : {16, 8, 4, 2}) {
    LSOP_HIP(launch_cols<T>(op->lx, tmp, Dt<T>::gs(op), op->nx, op->pz(), m, false, Dt<T>::twx(op), s, tile));
    LSOP_HIP(hipEventRecord(a, s));
    for (int rep = 0; rep < 3; ++rep)
      LSOP_HIP(launch_cols<T>(op->lx, tmp, Dt<T>::gs(op), op->nx, op->pz(), m, false, Dt<T>::twx(op), s, tile));
    LSOP_HIP(hipEventRecord(b, s));
    LSOP_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    LSOP_HIP(hipEventElapsedTime(&ms, a, b));
    if (ms < best * 0.98f) {
      best = ms;
      best_tile = tile;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  op->col_tile = best_tile;
  return LSOP_OK;
}

int check_op(const lsop_op* op) {
  if (!op) return fail(LSOP_EINVAL, "null operator handle");
  if (!op->ready) return fail(LSOP_EINVAL, "lsop_set_problem has not been called");
  return LSOP_OK;
}

// ---------------------------------------------------------- preconditioner
// Orthonormal basis of the r columns (probe-major rows of n elements) of Y,
// independently on each segment of `seg` elements (seg = n: the whole range),
// written to Q; Y is overwritten.  Columns are taken in blocks of 64: each
// block is first projected out of the previous blocks' basis twice (block
// classical Gram-Schmidt), then orthonormalised by Cholesky-QR run twice in the
// metric of its FP64 Gram matrix.  A column is dropped (numerically
// dependent) when its remaining norm falls below a fixed fraction of its norm
// before any projection (its squared norm per segment, written to R as FP64
// reals).  G, X, R: FP64 scratch of nseg * r * 64 entries each;
// kept[(block) * nseg + sg] receives the kept column counts of the final pass.
// full = false (an intermediate basis of the power iteration, whose only use is
// the next sample: its span matters, not how orthonormal it is) projects once
// and runs Cholesky-QR once.
template <typename T>
int orth_blocks(Cx<T>* Y, Cx<T>* Q, int r, size_t n, size_t seg, int nseg, int ksub, Cx<double>* G, Cx<double>* X,
                Cx<double>* R, Cx<double>* part, size_t part_cap, int* kept, hipStream_t s, bool full = true) {
  constexpr int B = 64;
  const int passes = full ? 2 : 1;
  const double tol = std::is_same<T, float>::value ? 1e-9 : 1e-24;
  const double e = sizeof(Cx<T>);
  for (int c0 = 0; c0 < r; c0 += B) {
    const int kb = std::min(B, r - c0);
    Cx<T>* Yb = Y + (size_t)c0 * n;
    Cx<T>* Qb = Q + (size_t)c0 * n;
    if (c0 > 0) {  // squared column norms of the block before projection, per segment (the drop test's reference)
      LSOP_HIP(prof("orth_norms", fn_name("k_seg_colnorm2", tname<T>()), (double)kb * n * e, 4.0 * kb * (double)n, kb,
                    s, [&] {
                      return launch_seg_colnorm2<T>(Yb, kb, n, seg, nseg, reinterpret_cast<double*>(R), s);
                    }));
    }
    for (int pass = 0; pass < passes && c0 > 0; ++pass) {
      LSOP_HIP(p_ah_b<T>("orth_project", Q, c0, Yb, nullptr, kb, n, seg, G, part, ksub, s, -1.0, part_cap));
      LSOP_HIP(p_update<T>("orth_project", Q, c0, G, (size_t)c0 * kb, kb, Yb, nullptr, 0.0, Yb, nullptr, n, seg, s));
    }
    for (int pass = 0; pass < passes; ++pass) {
      const Cx<T>* src = pass == 0 ? Yb : Qb;
      Cx<T>* dst = Qb;  // the second pass updates the first pass's basis in place (kb <= 64 vectors)
      LSOP_HIP(p_ah_b<T>("orth_gram", src, kb, src, nullptr, kb, n, seg, G, part, ksub, s, 1.0, part_cap));
      LSOP_HIP(prof("orth_coeffs", "k_gram_orth_lds", 2.0 * nseg * kb * kb * sizeof(Cx<double>),
                    8.0 / 3.0 * kb * kb * (double)kb * nseg, nseg, s, [&] {
                      return launch_gram_orth(G, X, kb, pass == 0 ? tol : 1e-6, kept + (c0 / B) * nseg, s, nseg,
                                              (pass == 0 && c0 > 0) ? reinterpret_cast<const double*>(R)
                                                                    : nullptr);
                    }));
      LSOP_HIP(p_update<T>("orth_update", src, kb, X, (size_t)kb * kb, kb, nullptr, nullptr, 0.0, dst, nullptr, n, seg,
                           s));
    }
  }
  return LSOP_OK;
}

// Q = orth(Y) over the whole grid (Alg. 2 step 3); Y is overwritten.
template <typename T>
int orth_impl(lsop_precond* pc, Cx<T>* Yin, Cx<T>* Qout, hipStream_t s) {
  const int r = pc->probes;
  const size_t n = pc->op->n();
  Cx<double>* G = pc->small;
  Cx<double>* X = G + (size_t)r * r;
  Cx<double>* R = X + (size_t)r * r;
  return orth_blocks<T>(Yin, Qout, r, n, n, 1, pc->ksplit, G, X, R, pc->part, pc->part_cap, pc->dflag, s);
}

template <typename T>
int build_impl(lsop_precond* pc, const double* omega, hipStream_t s) {
  lsop_op* op = pc->op;
  const int l = pc->probes, r = pc->rank;
  const size_t n = op->n();
  Cx<T>* U = reinterpret_cast<Cx<T>*>(pc->U);
  Cx<T>* W = reinterpret_cast<Cx<T>*>(pc->W);
  Cx<T>* Y = reinterpret_cast<Cx<T>*>(pc->Y);
  // Alg. 2 step 1: Gaussian probes
  if (omega) LSOP_HIP(launch_real_to_complex<T>(omega, Y, (size_t)l * n, s));
  else LSOP_HIP(launch_philox_normal<T>(Y, l, n, pc->seed, s));
  // step 2: Y0 = G0 (V Omega)
  int st = apply_impl<T>(op, LSOP_MODE_G0V, Y, Y, nullptr, nullptr, nullptr, l, s);
  if (st) return st;
  // step 3: Q0 = orth(Y0)
  if ((st = orth_impl<T>(pc, Y, U, s))) return st;
  // step 4: power iterations with the adjoint
  for (int j = 0; j < pc->q; ++j) {
    if ((st = apply_impl<T>(op, LSOP_MODE_VHG0H, U, Y, nullptr, nullptr, nullptr, l, s))) return st;
    if ((st = orth_impl<T>(pc, Y, W, s))) return st;  // W holds Q~_j
    if ((st = apply_impl<T>(op, LSOP_MODE_G0V, W, Y, nullptr, nullptr, nullptr, l, s))) return st;
    if ((st = orth_impl<T>(pc, Y, U, s))) return st;
  }
  // step 5: W = V^H G0^H Q_q, U = Q_q
  if ((st = apply_impl<T>(op, LSOP_MODE_VHG0H, U, W, nullptr, nullptr, nullptr, l, s))) return st;
  int flags[34] = {0};
  if (l > r) {
    // oversampled: G0 V ~= Q W~^H with l columns; W~ = Q2 R2, R2^H = U_b S V_b^H (FP64 SVD),
    // U = Q (U_b S)(:, :r), W = Q2 V_b(:, :r)
    Cx<T>* Q2 = reinterpret_cast<Cx<T>*>(pc->Q2);
    LSOP_HIP(hipMemcpyAsync(Y, W, sizeof(Cx<T>) * (size_t)l * n, hipMemcpyDeviceToDevice, s));
    if ((st = orth_impl<T>(pc, Y, Q2, s))) return st;
    Cx<double>* R2 = pc->svdw;
    Cx<double>* Bc = R2 + (size_t)l * l;
    Cx<double>* Vc = Bc + (size_t)l * l;
    Cx<double>* Mu = Vc + (size_t)l * l;
    Cx<double>* Mw = Mu + (size_t)l * r;
    LSOP_HIP(p_gemm_ah_b<T>(Q2, l, W, nullptr, l, n, R2, pc->part, pc->ksplit, s, pc->part_cap));
    LSOP_HIP(hipMemsetAsync(pc->dflag + 33, 0, sizeof(int), s));
    LSOP_HIP(prof("lowrank_truncate", "k_svd_jacobi", 5.0 * l * l * sizeof(Cx<double>), 0.0, l, s,
                  [&] { return launch_svd_trunc(R2, l, r, Bc, Vc, Mu, Mw, pc->dflag + 33, s); }));
    LSOP_HIP(p_gemm_update<T>(U, l, Mu, r, nullptr, nullptr, 0.0, Y, nullptr, n, s));
    LSOP_HIP(p_gemm_update<T>(Q2, l, Mw, r, nullptr, nullptr, 0.0, W, nullptr, n, s));
    LSOP_HIP(hipMemcpyAsync(U, Y, sizeof(Cx<T>) * (size_t)r * n, hipMemcpyDeviceToDevice, s));
  }
  // eq. (12): Z = (I_r - W^H U)^{-1}
  Cx<double>* M = pc->small;
  Cx<double>* work = M + (size_t)r * r;
  LSOP_HIP(p_gemm_ah_b<T>(W, r, U, nullptr, r, n, M, pc->part, pc->ksplit, s, pc->part_cap));
  LSOP_HIP(hipMemsetAsync(pc->dflag + 32, 0, sizeof(int), s));
  LSOP_HIP(launch_lu_inverse_i_minus(M, pc->Z, work, r, pc->dflag + 32, s));
  LSOP_HIP(hipMemcpyAsync(flags, pc->dflag, sizeof(flags), hipMemcpyDeviceToHost, s));
  LSOP_HIP(hipStreamSynchronize(s));
  pc->kept = 0;
  if (l > r) {
    pc->kept = flags[33];
  } else {
    for (int b = 0; b < (l + 63) / 64; ++b) pc->kept += flags[b];
  }
  if (flags[32]) return fail(LSOP_ESINGULAR, "I - W^H U is numerically singular");
  pc->built = true;
  return LSOP_OK;
}

template <typename T>
int hodlr_apply(lsop_precond* pc, const Cx<T>* x, const int* xidx, Cx<T>* y, const int* yidx, int nvec, int upto,
                hipStream_t s);

// y = x + U Z W^H x  (or, when series_update, psi <- psi - r - U Z W^H r with x = r, y = psi);
// HODLR: y = A_h^{-1} x (or psi <- psi - A_h^{-1} r)
template <typename T>
int pc_apply_impl(lsop_precond* pc, const Cx<T>* x, Cx<T>* y, const int* vidx, int nvec, bool series_update,
                  hipStream_t s) {
  const size_t n = pc->op->n();
  if (pc->kind == LSOP_PC_IDENTITY) {
    if (series_update) return launch_axpby<T>(x, y, -1.0, 1.0, vidx, nvec, n, s) == hipSuccess
                                  ? LSOP_OK
                                  : fail(LSOP_EHIP, "axpby launch failed");
    if (x != y) {
      if (vidx) {
        LSOP_HIP(launch_axpby<T>(x, y, 1.0, 0.0, vidx, nvec, n, s));
      } else {
        LSOP_HIP(hipMemcpyAsync(y, x, sizeof(Cx<T>) * n * nvec, hipMemcpyDeviceToDevice, s));
      }
    }
    return LSOP_OK;
  }
  if (pc->kind == LSOP_PC_GAMMA) {  // H = gamma = i V_eps / eps pointwise (convergent Born series)
    const lsop_op* op = pc->op;
    if (!op->damped) return fail(LSOP_EINVAL, "H = gamma needs an operator set by lsop_set_problem_damped");
    const Cx<T>* V = reinterpret_cast<const Cx<T>*>(std::is_same<T, float>::value ? (const void*)op->v32
                                                                                    : (const void*)op->v64);
    const hipError_t e = launch_vmul<T>(V, x, vidx, nullptr, y, vidx, nvec, n, series_update ? 4 : 3, 1.0 / op->eps, s);
    return e == hipSuccess ? LSOP_OK : fail(LSOP_EHIP, "gamma launch failed");
  }
  if (pc->kind == LSOP_PC_SCALAR) {  // H = alpha I: y = alpha x, or psi <- psi - alpha r
    const hipError_t e = series_update ? launch_axpby<T>(x, y, -pc->alpha, 1.0, vidx, nvec, n, s)
                                       : launch_axpby<T>(x, y, pc->alpha, 0.0, vidx, nvec, n, s);
    return e == hipSuccess ? LSOP_OK : fail(LSOP_EHIP, "axpby launch failed");
  }
  if (pc->kind == LSOP_PC_HODLR) {
    if (!series_update) return hodlr_apply<T>(pc, x, vidx, y, vidx, nvec, 0, s);
    // psi <- psi - H r, H r into the compact temporary chunk by chunk
    Cx<T>* hy = reinterpret_cast<Cx<T>*>(pc->hy);
    for (int c = 0; c < nvec; c += pc->tcap) {
      const int m = std::min(pc->tcap, nvec - c);
      const int* vc = vidx ? vidx + c : nullptr;
      const Cx<T>* xc = vidx ? x : x + (size_t)c * n;
      Cx<T>* yc = vidx ? y : y + (size_t)c * n;
      int st = hodlr_apply<T>(pc, xc, vc, hy, nullptr, m, 0, s);
      if (st) return st;
      LSOP_HIP(launch_axpy_map<T>(hy, yc, vc, -1.0, m, n, s));
    }
    return LSOP_OK;
  }
  const int r = pc->rank;
  const Cx<T>* U = reinterpret_cast<const Cx<T>*>(pc->U);
  const Cx<T>* W = reinterpret_cast<const Cx<T>*>(pc->W);
  Cx<double>* T1 = pc->small + 3 * (size_t)r * r;
  Cx<double>* T2 = T1 + (size_t)r * pc->tcap;
  for (int c = 0; c < nvec; c += pc->tcap) {
    const int m = std::min(pc->tcap, nvec - c);
    const int* vc = vidx ? vidx + c : nullptr;
    const size_t off = vidx ? 0 : (size_t)c * n;
    LSOP_HIP(p_gemm_ah_b<T>(W, r, x + off, vc, m, n, T1, pc->part, pc->ksplit, s, pc->part_cap));
    LSOP_HIP(launch_small_gemm(pc->Z, T1, T2, r, m, series_update ? -1.0 : 1.0, s));
    if (series_update)
      LSOP_HIP(p_gemm_update<T>(U, r, T2, m, y + off, x + off, -1.0, y + off, vc, n, s));
    else
      LSOP_HIP(p_gemm_update<T>(U, r, T2, m, x + off, nullptr, 0.0, y + off, vc, n, s));
  }
  return LSOP_OK;
}

// ------------------------------------------------------------------ HODLR
// Section 2.4.  Level l (0 = root) has 2^l nodes of width nx >> l grid
// columns; a node's halves are segments of (width / 2) * nz consecutive cells.
// A_l = A_{l+1} - Ut_l Vt_l^H, where A_levels is the block diagonal of dense
// leaves and Ut_l Vt_l^H holds the off-diagonal blocks of the level's nodes:
// with G0 V[I1, I2] ~= Q12 v12^H (Alg. 1, q = 0; v12 = (G0 V[I1, I2])^H Q12),
// Ut = diag(Q12, Q21) and Vt^H = [[0, v12^H], [v21^H, 0]].  Both are stored
// packed as full-grid arrays (Q: Q12 on I1 cells and Q21 on I2 cells; V: v12
// on I2 and v21 on I1).  Woodbury gives
//   A_l^{-1} y = A_{l+1}^{-1} y + Wp K^{-1} Vt^H A_{l+1}^{-1} y,
//   Wp = A_{l+1}^{-1} Ut,  K = I - Vt^H Wp = [[I, -v12^H w2], [-v21^H w1, I]],
// applied bottom-up from the leaf solve.

template <typename T>
const Cx<T>* lev_gs(const hodlr_level& L);
template <>
const Cx<float>* lev_gs<float>(const hodlr_level& L) { return L.gs32; }
template <>
const Cx<double>* lev_gs<double>(const hodlr_level& L) { return L.gs64; }
template <typename T>
const Cx<T>* lev_tw(const hodlr_level& L);
template <>
const Cx<float>* lev_tw<float>(const hodlr_level& L) { return L.tw32; }
template <>
const Cx<double>* lev_tw<double>(const hodlr_level& L) { return L.tw64; }

// partial chunks per segment for the block-diagonal inner products
int hodlr_ksub(const lsop_precond* pc, size_t seg, int nseg) {
  const int want = (int)std::max<size_t>(1, (seg + 4095) / 4096);
  return std::max(1, std::min(want, pc->ksub_cap / nseg));
}

// Sub-domain convolution at level lv: y = G0 V x (adj = false) or
// V^H G0^H x (adj = true) on each node's strip alone, input restricted to the
// half in_half of every node, only the half out_half of y written.
//
// Levels marked half move only the input half through the intermediate and convolve at period W (the node
// width) in x: the input half's h = W / 2 rows go to the first half of the period and the output half is read
// from the second, so the circular lag (period position of the output minus that of the input) runs over
// 1 .. W - 1 and never wraps.  The forward table puts lag c at position c; the adjoint pass multiplies by the
// conjugate spectrum, i.e. the table conj(K(W - c)).  The strip rows are mapped to period positions so that the
// circular lag equals |x_out - x_in| (forward) or W - |x_out - x_in| (adjoint); for input position i and output
// position h + j (0 <= i, j < h):
//   forward, half 0 -> 1:  x_in = i,         x_out = h + j
//   forward, half 1 -> 0:  x_in = W - 1 - i, x_out = h - 1 - j
//   adjoint, half 0 -> 1:  x_in = h - 1 - i, x_out = W - 1 - j
//   adjoint, half 1 -> 0:  x_in = h + i,     x_out = j
// (G0 depends on |x_out - x_in| only, Section 2.2.)
template <typename T>
int hodlr_subconv(lsop_precond* pc, int lv, bool adj, const Cx<T>* x, Cx<T>* y, int nvec, int in_half, int out_half,
                  hipStream_t s) {
  lsop_op* op = pc->op;
  const hodlr_level& L = pc->lev[lv];
  const int W = L.width, nodes = op->nx / W, half = W / 2;
  const int in_lo = in_half ? half : 0, in_hi = in_half ? W : half;
  const int out_lo = out_half ? half : 0, out_hi = out_half ? W : half;
  if (L.half && in_half == out_half) return fail(LSOP_EINVAL, "sub-domain convolution within one half");
  RowMap rin, rout;
  int rows = W;  // rows per node in the intermediate
  if (L.half) {
    rows = half;
    rin.ns = rout.ns = half;
    if (!adj) {
      rin.xa = in_half ? W - 1 : 0, rin.xs = in_half ? -1 : 1;
      rout.xa = in_half ? half - 1 : half, rout.xs = in_half ? -1 : 1;
    } else {
      rin.xa = in_half ? half : half - 1, rin.xs = in_half ? 1 : -1;
      rout.xa = in_half ? 0 : W - 1, rout.xs = in_half ? 1 : -1;
    }
  }
  const size_t n = op->n();
  Cx<T>* tmp = reinterpret_cast<Cx<T>*>(op->tmp);
  const double e = sizeof(Cx<T>), nn = (double)n, np = (double)nodes * rows * op->pz();
  for (int c = 0; c < nvec; c += op->max_vec) {
    const int m = std::min(op->max_vec, nvec - c);
    const size_t off = (size_t)c * n;
    std::string fcol;
    LSOP_HIP(prof("hodlr_rows_fwd", fn_name("k_rows_fwd", tname<T>(), op->lz), m * (0.5 * nn * e + np * e), 0.0, m, s, [&] {
      return launch_rows_fwd<T>(op->lz, x + off, Dt<T>::chi(op), tmp, nullptr, W, op->nz, m * nodes, !adj,
                                Dt<T>::twz(op), s, nodes, in_lo, in_hi, nullptr, rows, rin);
    }));
    LSOP_HIP(prof("hodlr_cols", fcol, m * 2.0 * np * e + 2.0 * op->pz() * L.lx * e, 0.0, m, s, [&] {
      int used = 0;
      hipError_t er = launch_cols<T>(L.lx, tmp, lev_gs<T>(L), rows, op->pz(), m * nodes, adj, lev_tw<T>(L), s, 0,
                                     &used);
      fcol = L.lx == 1 ? fn_name("k_cols_len1", tname<T>()) : fn_name("k_cols", tname<T>(), L.lx, used);
      return er;
    }));
    LSOP_HIP(prof("hodlr_rows_inv", fn_name("k_rows_inv", tname<T>(), op->lz), m * (np * e + 0.5 * nn * e), 0.0, m, s,
                  [&] {
      return launch_rows_inv<T>(op->lz, tmp, x + off, Dt<T>::chi(op), nullptr, y + off, nullptr, nullptr, W, op->nz,
                                m * nodes, adj ? 3 : 1, Dt<T>::twz(op), s, nodes, out_lo, out_hi, nullptr, rows, rout);
    }));
  }
  return LSOP_OK;
}

// FP64 workspace of one orthonormalisation (orth_blocks): G, X, R, the split-K partials and the kept counts.
struct OrthScratch {
  Cx<double>*G, *X, *R, *part;
  size_t part_cap;
  int* kept;
};

// Orthonormal bases, separately on every half-node segment of level lv.
template <typename T>
int hodlr_orth(lsop_precond* pc, int lv, Cx<T>* Yin, Cx<T>* Qout, const OrthScratch& sc, hipStream_t s, bool full) {
  const int W = pc->lev[lv].width, nseg = 2 * (pc->op->nx / W);
  const size_t seg = (size_t)(W / 2) * pc->op->nz;
  return orth_blocks<T>(Yin, Qout, pc->rank, pc->op->n(), seg, nseg, hodlr_ksub(pc, seg, nseg), sc.G, sc.X, sc.R,
                        sc.part, sc.part_cap, sc.kept, s, full);
}

// Sampling of level lv (Alg. 1 on both off-diagonal blocks of every node, q power iterations): the
// orthonormal bases U, returned in Y, and the right factors V (lev[lv].V).  Q and sc are workspace; the FFT
// passes use the operator's intermediate.
template <typename T>
int hodlr_sample(lsop_precond* pc, int lv, const double* omega, Cx<T>* Y, Cx<T>* Q, const OrthScratch& sc,
                 hipStream_t s) {
  const int r = pc->rank;
  const size_t n = pc->op->n();
  Cx<T>* V = reinterpret_cast<Cx<T>*>(pc->lev[lv].V);
  int st;
  // Alg. 1 step 1: Gaussian probes of this level
  if (omega) LSOP_HIP(launch_real_to_complex<T>(omega + (size_t)lv * r * n, Y, (size_t)r * n, s));
  else LSOP_HIP(launch_philox_normal<T>(Y, r, n, pc->seed, s, lv * r));
  // step 2: samples of both off-diagonal blocks of every node, G0 V[I1, I2] Om
  // on the I1 cells and G0 V[I2, I1] Om on the I2 cells
  if ((st = hodlr_subconv<T>(pc, lv, false, Y, Q, r, 1, 0, s))) return st;
  if ((st = hodlr_subconv<T>(pc, lv, false, Y, Q, r, 0, 1, s))) return st;
  // step 3: orthonormal bases per half-node (result in Y); with power iterations this basis is an
  // intermediate one (one projection and one Cholesky-QR pass), the last one is orthonormalised in full
  const int q = lv >= pc->q_from ? pc->q : 0;
  if ((st = hodlr_orth<T>(pc, lv, Q, Y, sc, s, q == 0))) return st;
  // optional power iterations (Alg. 1 step 4) on both blocks of every node
  for (int j = 0; j < q; ++j) {
    if ((st = hodlr_subconv<T>(pc, lv, true, Y, Q, r, 0, 1, s))) return st;
    if ((st = hodlr_subconv<T>(pc, lv, true, Y, Q, r, 1, 0, s))) return st;
    if ((st = hodlr_orth<T>(pc, lv, Q, Y, sc, s, false))) return st;
    if ((st = hodlr_subconv<T>(pc, lv, false, Y, Q, r, 1, 0, s))) return st;
    if ((st = hodlr_subconv<T>(pc, lv, false, Y, Q, r, 0, 1, s))) return st;
    if ((st = hodlr_orth<T>(pc, lv, Q, Y, sc, s, j == q - 1))) return st;
  }
  // right factors v12 = (G0 V[I1, I2])^H Q12 on I2, v21 on I1
  if ((st = hodlr_subconv<T>(pc, lv, true, Y, V, r, 0, 1, s))) return st;
  if ((st = hodlr_subconv<T>(pc, lv, true, Y, V, r, 1, 0, s))) return st;
  return LSOP_OK;
}

// In-place inverse of the m x m block at offset o of each of cnt FP64
// matrices (leading dimension ld, batch stride st) by the 2 x 2 block formula
// of Section 2.4: with X = A^{-1} and S = D - C X B,
//   [[A, B], [C, D]]^{-1} = [[X + X B S^{-1} C X, -X B S^{-1}], [-S^{-1} C X, S^{-1}]],
// recursing on A and S down to 64 x 64 blocks (Gauss-Jordan with partial
// pivoting; flags[b] set on a vanishing pivot).  Temporaries of recursion
// depth d at tbase + toff[d] (block_inverse_temps).
// W: the working precision (double, or float for the leaves of a complex-FP32 preconditioner).
template <typename W>
int block_inverse(Cx<W>* M, size_t ld, size_t st, int cnt, size_t o, int m, int depth, Cx<W>* tbase,
                  const std::vector<size_t>& toff, int* flags, hipStream_t s) {
  if (m <= 64) {
    LSOP_HIP(prof("block_inv_base", fn_name("k_lu_inverse_lds", tname<W>()), 2.0 * m * m * (double)sizeof(Cx<W>) * cnt,
                  8.0 * m * m * (double)m * cnt, cnt, s, [&] {
      if constexpr (std::is_same<W, double>::value)
        return launch_lu_inverse(M + o, ld, st, M + o, ld, st, nullptr, m, true, flags, cnt, s);
      else
        return launch_lu_inverse_small_f32(M + o, ld, st, M + o, ld, st, m, true, flags, cnt, s);
    }));
    return LSOP_OK;
  }
  const int h = m / 2, h2 = m - h;
  const size_t A = o, B = o + h, C = o + (size_t)h * ld, D = C + h;
  Cx<W>* T1 = tbase + toff[depth];         // h x h2
  Cx<W>* T2 = T1 + (size_t)cnt * h * h2;   // h2 x h
  const size_t s1 = (size_t)h * h2;
  int rc = block_inverse<W>(M, ld, st, cnt, A, h, depth + 1, tbase, toff, flags, s);
  if (rc) return rc;
  auto gemm = [&](const Cx<W>* a, size_t lda, size_t sa, const Cx<W>* b, size_t ldb, size_t sb, Cx<W>* c, size_t ldc,
                  size_t sc, int mm, int nn, int kk, double alpha, double beta) {
    return p_bgemm<W>("block_inv_gemm", a, lda, sa, b, ldb, sb, c, ldc, sc, nullptr, nullptr, mm, nn, kk, alpha, beta,
                      cnt, s);
  };
  LSOP_HIP(gemm(M + A, ld, st, M + B, ld, st, T1, h2, s1, h, h2, h, 1.0, 0.0));      // T1 = X B
  LSOP_HIP(gemm(M + C, ld, st, T1, h2, s1, M + D, ld, st, h2, h2, h, -1.0, 1.0));    // D <- S = D - C X B
  rc = block_inverse<W>(M, ld, st, cnt, D, h2, depth + 1, tbase, toff, flags, s);   // D <- S^{-1}
  if (rc) return rc;
  LSOP_HIP(gemm(M + C, ld, st, M + A, ld, st, T2, h, s1, h2, h, h, 1.0, 0.0));      // T2 = C X
  LSOP_HIP(gemm(T1, h2, s1, M + D, ld, st, M + B, ld, st, h, h2, h2, -1.0, 0.0));   // B <- -X B S^{-1}
  LSOP_HIP(gemm(M + B, ld, st, T2, h, s1, M + A, ld, st, h, h, h2, -1.0, 1.0));     // A <- X + X B S^{-1} C X
  LSOP_HIP(gemm(M + D, ld, st, T2, h, s1, M + C, ld, st, h2, h, h2, -1.0, 0.0));    // C <- -S^{-1} C X
  return LSOP_OK;
}

// offsets (from the temporaries' base) of each recursion depth of block_inverse on m0 x m0 blocks
std::vector<size_t> block_inverse_temps(int m0, int cnt, size_t* total) {
  std::vector<size_t> off;
  size_t at = 0;
  for (int m = m0; m > 64; m = (m + 1) / 2) {
    off.push_back(at);
    const size_t h2 = (size_t)(m - m / 2);
    at += 2 * (size_t)cnt * h2 * h2;
  }
  off.push_back(at);
  *total = at;
  return off;
}

template <typename T>
int hodlr_leaves(lsop_precond* pc, hipStream_t s) {
  lsop_op* op = pc->op;
  const int nl = pc->leaf_w * op->nz;
  Cx<T>* dinv = reinterpret_cast<Cx<T>*>(pc->dinv);
  for (int l0 = 0; l0 < pc->nleaf; l0 += pc->leaf_chunk) {
    const int cnt = std::min(pc->leaf_chunk, pc->nleaf - l0);
    size_t total = 0;
    const std::vector<size_t> toff = block_inverse_temps(nl, cnt, &total);
    LSOP_HIP(hipMemsetAsync(pc->hflag, 0, sizeof(int) * cnt, s));
    // complex-FP32 preconditioners invert their leaves in FP32 (error ~ cond * 1e-7, far below the low-rank
    // truncation of the off-diagonal blocks); complex-FP64 ones in FP64
    int rc;
    if constexpr (std::is_same<T, float>::value) {
      Cx<float>* lw = reinterpret_cast<Cx<float>*>(pc->lwork);
      LSOP_HIP(launch_leaf_form<float>(op->ktab, op->chi64, lw, op->nz, nl, l0, cnt, s));
      rc = block_inverse<float>(lw, nl, (size_t)nl * nl, cnt, 0, nl, 0, lw + (size_t)cnt * nl * nl, toff, pc->hflag, s);
    } else {
      LSOP_HIP(launch_leaf_form<double>(op->ktab, op->chi64, pc->lwork, op->nz, nl, l0, cnt, s));
      rc = block_inverse<double>(pc->lwork, nl, (size_t)nl * nl, cnt, 0, nl, 0, pc->lwork + (size_t)cnt * nl * nl,
                                 toff, pc->hflag, s);
    }
    if (rc) return rc;
    std::vector<int> flags(cnt, 0);
    LSOP_HIP(hipMemcpyAsync(flags.data(), pc->hflag, sizeof(int) * cnt, hipMemcpyDeviceToHost, s));
    LSOP_HIP(hipStreamSynchronize(s));
    for (int f : flags)
      if (f) return fail(LSOP_ESINGULAR, "a HODLR leaf block is numerically singular");
    if constexpr (std::is_same<T, float>::value)
      LSOP_HIP(launch_transpose_f32(reinterpret_cast<const Cx<float>*>(pc->lwork), dinv + (size_t)l0 * nl * nl, nl,
                                    cnt, s));
    else
      LSOP_HIP(launch_transpose_convert<T>(pc->lwork, dinv + (size_t)l0 * nl * nl, nl, cnt, s));
  }
  return LSOP_OK;
}

// y = A_upto^{-1} x for nvec vectors: x rows through xidx, y rows through yidx
// (NULL: consecutive).  upto = 0 is the full preconditioner.
template <typename T>
int hodlr_apply(lsop_precond* pc, const Cx<T>* x, const int* xidx, Cx<T>* y, const int* yidx, int nvec, int upto,
                hipStream_t s) {
  lsop_op* op = pc->op;
  const size_t n = op->n();
  const int r = pc->rank, nl = pc->leaf_w * op->nz;
  const Cx<T>* dinv = reinterpret_cast<const Cx<T>*>(pc->dinv);
  const double e = sizeof(Cx<T>);
  for (int c = 0; c < nvec; c += pc->tcap) {
    const int m = std::min(pc->tcap, nvec - c);
    const int* xc = xidx ? xidx + c : nullptr;
    const int* yc = yidx ? yidx + c : nullptr;
    const Cx<T>* xb = xidx ? x : x + (size_t)c * n;
    Cx<T>* yb = yidx ? y : y + (size_t)c * n;
    // leaves: y_k = D_k^{-1} x_k (D_k^{-1} stored transposed: y = x D^{-T})
    LSOP_HIP(p_bgemm<T>("hodlr_leaf_apply", xb, n, nl, dinv, nl, (size_t)nl * nl, yb, n, nl, xc, yc, m, nl, nl, 1.0,
                        0.0, pc->nleaf, s));
    for (int lv = pc->levels - 1; lv >= upto; --lv) {
      const hodlr_level& L = pc->lev[lv];
      const int nodes = op->nx / L.width, nseg = 2 * nodes;
      const size_t seg = (size_t)(L.width / 2) * op->nz;
      const int ksub = hodlr_ksub(pc, seg, nseg);
      const Cx<T>* V = reinterpret_cast<const Cx<T>*>(L.V);
      const Cx<T>* Wp = reinterpret_cast<const Cx<T>*>(L.Wp);
      if constexpr (std::is_same<T, float>::value) {
        // the update rounds the core's output to FP32 anyway: the core product runs on the fp32 matrix cores
        // (K^{-1} inverted in FP64, applied from its FP32 copy) on the inner products summed in FP64 and rounded
        // to FP32 by their reduction
        LSOP_HIP(p_ah_b<T>("hodlr_apply_ah_b", V, r, yb, yc, m, n, seg, pc->hG, pc->part, ksub, s, 1.0,
                           pc->part_cap, pc->hG32));
        LSOP_HIP(p_bgemm<float>("hodlr_core_apply", L.kinv32, 2 * r, (size_t)4 * r * r, pc->hG32, m,
                                (size_t)2 * r * m, pc->hX32, m, (size_t)2 * r * m, nullptr, nullptr, 2 * r, m, 2 * r,
                                1.0, 0.0, nodes, s));
        // the update takes the cores' FP32 products as they are (an FP64 copy would hold the same values)
        LSOP_HIP(p_update<T, float>("hodlr_apply_update", Wp, r, pc->hX32, (size_t)r * m, m, yb, nullptr, 0.0, yb, yc,
                                    n, seg, s));
      } else {
        LSOP_HIP(p_ah_b<T>("hodlr_apply_ah_b", V, r, yb, yc, m, n, seg, pc->hG, pc->part, ksub, s, 1.0,
                           pc->part_cap));
        LSOP_HIP(p_bgemm<double>("hodlr_core_apply", L.kinv, 2 * r, (size_t)4 * r * r, pc->hG, m, (size_t)2 * r * m,
                                 pc->hX, m, (size_t)2 * r * m, nullptr, nullptr, 2 * r, m, 2 * r, 1.0, 0.0, nodes, s));
        LSOP_HIP(p_update<T>("hodlr_apply_update", Wp, r, pc->hX, (size_t)r * m, m, yb, nullptr, 0.0, yb, yc, n, seg,
                             s));
      }
    }
  }
  return LSOP_OK;
}

// kinv = K^{-1} P for every node of level lv, from G[sg] = V_sg^H Wp_sg
// (FP64, G0 = G[2k] on the first half, G1 = G[2k+1] on the second):
// K = [[I, -G1], [-G0, I]], S = I - G0 G1,
// K^{-1} = [[I + G1 S^{-1} G0, G1 S^{-1}], [S^{-1} G0, S^{-1}]],
// and P swaps the two column halves (the segment order of the products).
// S^{-1} by the recursive block formula, checked by max |S S^{-1} - I|; a
// node that fails the check is redone by Gauss-Jordan with pivoting.
int hodlr_core_inverse(lsop_precond* pc, int lv, hipStream_t s) {
  hodlr_level& L = pc->lev[lv];
  const int r = pc->rank, nodes = pc->op->nx / L.width;
  const size_t r2 = (size_t)r * r, ld = 2 * (size_t)r, st = 4 * r2;
  Cx<double>* K = L.kinv;
  Cx<double>* B00 = K;
  Cx<double>* B01 = K + r;
  Cx<double>* B10 = K + (size_t)r * ld;
  Cx<double>* B11 = B10 + r;
  const Cx<double>* G0 = pc->hG;
  const Cx<double>* G1 = pc->hG + r2;
  Cx<double>* Sc = pc->hX;  // copy of S, r x r per node
  size_t ttot = 0;
  const std::vector<size_t> toff = block_inverse_temps(r, nodes, &ttot);
  Cx<double>* tbase = pc->hK;
  Cx<double>* P = pc->hK + ttot;
  Cx<double>* gjw = P + (size_t)nodes * r2;
  double* dev = reinterpret_cast<double*>(pc->part);
  auto gemm = [&](const Cx<double>* a, size_t lda, size_t sa, const Cx<double>* b, size_t ldb, size_t sb,
                  Cx<double>* c, size_t ldc, size_t sc, double alpha, double beta) {
    return p_bgemm<double>("hodlr_core_gemm", a, lda, sa, b, ldb, sb, c, ldc, sc, nullptr, nullptr, r, r, r, alpha,
                           beta, nodes, s);
  };
  LSOP_HIP(launch_set_identity(B10, ld, st, r, nodes, s));
  LSOP_HIP(gemm(G0, r, 2 * r2, G1, r, 2 * r2, B10, ld, st, -1.0, 1.0));   // S = I - G0 G1
  LSOP_HIP(launch_set_identity(Sc, r, r2, r, nodes, s));
  LSOP_HIP(gemm(G0, r, 2 * r2, G1, r, 2 * r2, Sc, r, r2, -1.0, 1.0));
  LSOP_HIP(hipMemsetAsync(pc->hflag, 0, sizeof(int) * nodes, s));
  int rc = block_inverse(K, ld, st, nodes, (size_t)r * ld, r, 0, tbase, toff, pc->hflag, s);
  if (rc) return rc;
  LSOP_HIP(gemm(Sc, r, r2, B10, ld, st, P, r, r2, 1.0, 0.0));
  LSOP_HIP(launch_identity_deviation(P, r, r2, r, nodes, dev, s));
  std::vector<int> flags(nodes, 0);
  std::vector<double> devh(nodes, 0.0);
  LSOP_HIP(hipMemcpyAsync(flags.data(), pc->hflag, sizeof(int) * nodes, hipMemcpyDeviceToHost, s));
  LSOP_HIP(hipMemcpyAsync(devh.data(), dev, sizeof(double) * nodes, hipMemcpyDeviceToHost, s));
  LSOP_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < nodes; ++k) {
    if (!flags[k] && devh[k] <= 1e-8) continue;
    // pivoted Gauss-Jordan for this node
    LSOP_HIP(hipMemsetAsync(pc->hflag, 0, sizeof(int), s));
    LSOP_HIP(launch_lu_inverse(Sc + (size_t)k * r2, r, r2, B10 + (size_t)k * st, ld, st, gjw, r, true, pc->hflag, 1, s));
    int f = 0;
    LSOP_HIP(hipMemcpyAsync(&f, pc->hflag, sizeof(int), hipMemcpyDeviceToHost, s));
    LSOP_HIP(hipStreamSynchronize(s));
    if (f) return fail(LSOP_ESINGULAR, "a HODLR Woodbury core is numerically singular");
  }
  LSOP_HIP(gemm(G1, r, 2 * r2, B10, ld, st, B00, ld, st, 1.0, 0.0));       // G1 S^{-1}
  LSOP_HIP(launch_set_identity(B01, ld, st, r, nodes, s));
  LSOP_HIP(gemm(B00, ld, st, G0, r, 2 * r2, B01, ld, st, 1.0, 1.0));       // I + G1 S^{-1} G0
  LSOP_HIP(gemm(B10, ld, st, G0, r, 2 * r2, B11, ld, st, 1.0, 0.0));       // S^{-1} G0
  if (L.kinv32) LSOP_HIP(launch_convert<float, double>(K, L.kinv32, (size_t)nodes * st, s));
  return LSOP_OK;
}

// The levels are built deepest first: level lv's sampling needs only the operator, its solve (Wp =
// A_{lv+1}^{-1} U, then its node cores) the deeper levels.  (Sampling the next level on a second stream
// beside the current solve was measured: the FFT passes and the level GEMMs slowed each other down and the
// build gained 1.5%, so the build stays on one stream.)
template <typename T>
int hodlr_build(lsop_precond* pc, const double* omega, hipStream_t s) {
  lsop_op* op = pc->op;
  const int r = pc->rank;
  const size_t n = op->n();
  // build-only workspace: sampling buffers and the leaf workspace, taken from and returned to the
  // stream-ordered pool of stream s (no device-wide synchronisation, so builds on other streams keep running),
  // or carved from the operator's attached workspace (after the sub-domain spectra, which use its start as
  // their intermediate earlier on the same stream)
  const size_t bU = align_up(sizeof(Cx<T>) * r * n), bL = align_up(sizeof(Cx<double>) * pc->lwork_elems);
  struct Transient {
    lsop_precond* pc;
    hipStream_t s;
    bool pooled;
    ~Transient() {
      if (!pooled) {
        pc->U = pc->Y = nullptr;
        pc->lwork = nullptr;
        return;
      }
      for (void** p : {&pc->U, &pc->Y, reinterpret_cast<void**>(&pc->lwork)})
        if (*p) {
          (void)hipFreeAsync(*p, s);
          *p = nullptr;
        }
      (void)hipStreamSynchronize(s);
    }
  } transient{pc, s, !op->ws_external};
  if (op->ws_external) {
    if (op->scratch_bytes < 2 * bU + bL)
      return fail(LSOP_ENOMEM, "the attached workspace is smaller than the " + std::to_string(2 * bU + bL) +
                                   " bytes this HODLR build needs");
    char* w = reinterpret_cast<char*>(op->scratch);
    pc->U = w;
    pc->Y = w + bU;
    pc->lwork = reinterpret_cast<Cx<double>*>(w + 2 * bU);
  } else if (lib_malloc_async(&pc->U, sizeof(Cx<T>) * r * n, s) != hipSuccess ||
             lib_malloc_async(&pc->Y, sizeof(Cx<T>) * r * n, s) != hipSuccess ||
             lib_malloc_async(reinterpret_cast<void**>(&pc->lwork), sizeof(Cx<double>) * pc->lwork_elems, s) !=
                 hipSuccess) {
    (void)hipGetLastError();
    return fail(LSOP_ENOMEM, "HODLR build workspace allocation failed");
  }
  Cx<T>* Y = reinterpret_cast<Cx<T>*>(pc->Y);
  Cx<T>* Q = reinterpret_cast<Cx<T>*>(pc->U);
  const OrthScratch sc{pc->hG, pc->hX, pc->hK, pc->part, pc->part_cap, pc->hflag};
  // sub-domain spectra (depend on k0 and h)
  for (int lv = 0; lv < pc->levels; ++lv) {
    hodlr_level& L = pc->lev[lv];
    const size_t s1 = sizeof(Cx<double>) * (size_t)(2 * L.lx) * op->pz();
    int st = grow_scratch(op, s1);
    if (st) return st;
    LSOP_HIP(launch_spectrum(L.lx, op->lz, op->ktab, L.width, op->nz, reinterpret_cast<Cx<double>*>(op->scratch),
                             L.gs64, L.gs32, L.tw64, op->tw2z64, s, L.half));
  }
  int st = hodlr_leaves<T>(pc, s);
  if (st) return st;
  for (int lv = pc->levels - 1; lv >= 0; --lv) {
    hodlr_level& L = pc->lev[lv];
    const int nodes = op->nx / L.width, nseg = 2 * nodes;
    const size_t seg = (size_t)(L.width / 2) * op->nz;
    Cx<T>* V = reinterpret_cast<Cx<T>*>(L.V);
    Cx<T>* Wp = reinterpret_cast<Cx<T>*>(L.Wp);
    if ((st = hodlr_sample<T>(pc, lv, omega, Y, Q, sc, s))) return st;
    // Wp = A_{lv+1}^{-1} Ut
    if ((st = hodlr_apply<T>(pc, Y, nullptr, Wp, nullptr, r, lv + 1, s))) return st;
    // K per node from the per-half products V^H Wp, then kinv = K^{-1} P
    const int ksub = hodlr_ksub(pc, seg, nseg);
    LSOP_HIP(p_ah_b<T>("hodlr_core_ah_b", V, r, Wp, nullptr, r, n, seg, pc->hG, pc->part, ksub, s, 1.0, pc->part_cap));
    if ((st = hodlr_core_inverse(pc, lv, s))) return st;
  }
  pc->kept = r;
  pc->built = true;
  return LSOP_OK;
}

// Workspace of lsop_set_problem (the transposed FP64 intermediate of the spectrum) and of series_solve on nvec
// right-hand sides (the layouts carved in series_solve).
size_t spectrum_ws_bytes(const lsop_op* op) {
  return sizeof(Cx<double>) * (size_t)op->px() * op->py() * op->pz();
}

size_t series_ws_bytes(const lsop_op* op, int nvec, int init) {
  const size_t n = op->n();
  const size_t tail = align_up(sizeof(double) * nvec) + align_up(sizeof(int) * nvec);
  if (op->dtype != LSOP_MIXED) {
    const size_t esz = op->dtype == LSOP_C64 ? sizeof(Cx<float>) : sizeof(Cx<double>);
    return align_up(esz * n * nvec) * (init == LSOP_INIT_BEST ? 2 : 1) + tail;
  }
  // refinement (FP64 residual, FP32 right-hand side and correction, norms, list) and the inner series' residual
  return align_up(sizeof(Cx<double>) * n * nvec) + 3 * align_up(sizeof(Cx<float>) * n * nvec) + tail;
}

// --------------------------------------------------------------- series
// Runs eq. (11) on the vectors listed in `start` (all if empty).  rhs, psi, r
// are [nvec][n] buffers of T.  Per-vector results go to info[vi].
template <typename T>
int series_impl(lsop_op* op, lsop_precond* pc, const Cx<T>* rhs, Cx<T>* psi, int nvec, double tol, int max_iter,
                int init, const std::vector<int>& start, lsop_solve_info* info, Cx<T>* r, double* dnorm,
                int* dvidx, hipStream_t s, Cx<T>* alt = nullptr) {
  const size_t n = op->n();
  std::vector<int> active = start;
  if (active.empty())
    for (int v = 0; v < nvec; ++v) active.push_back(v);
  const int na0 = (int)active.size();
  LSOP_HIP(hipMemcpyAsync(dvidx, active.data(), sizeof(int) * na0, hipMemcpyHostToDevice, s));
  // ||rhs||^2
  std::vector<double> b2(nvec, 0.0), rn(nvec, 0.0);
  LSOP_HIP(launch_norm2<T>(rhs, dnorm, dvidx, na0, n, s));
  LSOP_HIP(hipMemcpyAsync(rn.data(), dnorm, sizeof(double) * na0, hipMemcpyDeviceToHost, s));
  LSOP_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < na0; ++k) b2[active[k]] = rn[k];
  // psi_0
  if (init == LSOP_INIT_H_RHS) {
    if (pc) {
      int st = pc_apply_impl<T>(pc, rhs, psi, dvidx, na0, false, s);
      if (st) return st;
    } else {
      LSOP_HIP(launch_axpby<T>(rhs, psi, 1.0, 0.0, dvidx, na0, n, s));
    }
  } else if (init == LSOP_INIT_ZERO) {
    LSOP_HIP(launch_axpby<T>(rhs, psi, 0.0, 0.0, dvidx, na0, n, s));
  } else if (init == LSOP_INIT_BEST) {
    // psi holds a candidate start: per vector, keep the better of it and H rhs (smaller residual)
    std::vector<double> nu(na0), nh(na0);
    LSOP_HIP(hipMemsetAsync(dnorm, 0, sizeof(double) * na0, s));
    int st = apply_impl<T>(op, LSOP_MODE_A, psi, r, rhs, dnorm, dvidx, na0, s);
    if (st) return st;
    LSOP_HIP(hipMemcpyAsync(nu.data(), dnorm, sizeof(double) * na0, hipMemcpyDeviceToHost, s));
    if (pc) {
      if ((st = pc_apply_impl<T>(pc, rhs, alt, dvidx, na0, false, s))) return st;
    } else {
      LSOP_HIP(launch_axpby<T>(rhs, alt, 1.0, 0.0, dvidx, na0, n, s));
    }
    LSOP_HIP(hipMemsetAsync(dnorm, 0, sizeof(double) * na0, s));
    if ((st = apply_impl<T>(op, LSOP_MODE_A, alt, r, rhs, dnorm, dvidx, na0, s))) return st;
    LSOP_HIP(hipMemcpyAsync(nh.data(), dnorm, sizeof(double) * na0, hipMemcpyDeviceToHost, s));
    LSOP_HIP(hipStreamSynchronize(s));
    std::vector<int> take;
    for (int k = 0; k < na0; ++k)
      if (!(nu[k] <= nh[k])) take.push_back(active[k]);  // also replaces a non-finite candidate
    if (!take.empty()) {
      LSOP_HIP(hipMemcpyAsync(dvidx, take.data(), sizeof(int) * take.size(), hipMemcpyHostToDevice, s));
      LSOP_HIP(launch_axpby<T>(alt, psi, 1.0, 0.0, dvidx, (int)take.size(), n, s));
      LSOP_HIP(hipStreamSynchronize(s));
    }
  }
  std::vector<double> prev(nvec, INFINITY);
  std::vector<int> rising(nvec, 0);
  for (int v : active) {
    info[v].iters = 0;
    info[v].status = LSOP_NOT_CONVERGED;
    info[v].rel_residual = INFINITY;
  }
  for (int it = 0;; ++it) {
    const int na = (int)active.size();
    LSOP_HIP(hipMemcpyAsync(dvidx, active.data(), sizeof(int) * na, hipMemcpyHostToDevice, s));
    LSOP_HIP(hipMemsetAsync(dnorm, 0, sizeof(double) * na, s));
    // eq. (13): a = psi - G0 V psi - psi0, with ||a||^2
    int st = apply_impl<T>(op, LSOP_MODE_A, psi, r, rhs, dnorm, dvidx, na, s);
    if (st) return st;
    LSOP_HIP(hipMemcpyAsync(rn.data(), dnorm, sizeof(double) * na, hipMemcpyDeviceToHost, s));
    LSOP_HIP(hipStreamSynchronize(s));
    std::vector<int> next;
    for (int k = 0; k < na; ++k) {
      const int v = active[k];
      const double rel = b2[v] > 0 ? std::sqrt(rn[k] / b2[v]) : std::sqrt(rn[k]);
      info[v].iters = it;
      info[v].rel_residual = rel;
      if (it == 0) info[v].rel_residual0 = rel;
      if (!std::isfinite(rel)) {
        info[v].status = LSOP_DIVERGED;
        continue;
      }
      if (rel <= tol) {
        info[v].status = LSOP_OK;
        continue;
      }
      rising[v] = rel > prev[v] ? rising[v] + 1 : 0;
      prev[v] = rel;
      if (rising[v] >= 5) {
        info[v].status = LSOP_DIVERGED;
        continue;
      }
      if (it == max_iter) {
        info[v].status = LSOP_NOT_CONVERGED;
        continue;
      }
      next.push_back(v);
    }
    active.swap(next);
    if (active.empty()) break;
    const int nn = (int)active.size();
    LSOP_HIP(hipMemcpyAsync(dvidx, active.data(), sizeof(int) * nn, hipMemcpyHostToDevice, s));
    // eq. (11): psi <- psi - H a
    if (pc) {
      st = pc_apply_impl<T>(pc, r, psi, dvidx, nn, true, s);
      if (st) return st;
    } else {
      LSOP_HIP(launch_axpby<T>(r, psi, -1.0, 1.0, dvidx, nn, n, s));
    }
  }
  return LSOP_OK;
}

// ------------------------------------------------------------------ GMRES
// Restarted GMRES(m) with right preconditioning, the Krylov method the paper compares the series with
// (Section 3.2.3): A H y = psi0 - A psi_start, psi = psi_start + H y.  Every right-hand side runs its own Arnoldi
// process (classical Gram-Schmidt, applied twice, FP64 sums) in lockstep with the others; the small Hessenberg
// least-squares problems are reduced by Givens rotations on the host in FP64.  A cycle ends for a right-hand side
// when its residual estimate reaches tol, at m inner iterations, at max_iter or on breakdown; the true residual
// A psi - psi0 then decides convergence (relative to ||psi0||, as the series).

// Workspace of gmres_impl: Krylov basis (m + 1 blocks of nvec vectors), two vector temporaries, the partial dot
// products, two coefficient columns, the solution coefficients, norms and the active list.
size_t gmres_ws_bytes(size_t n, int nvec, int m, size_t esz) {
  const size_t vb = align_up(esz * n * nvec);
  return (size_t)(m + 1) * vb + 2 * vb + align_up(sizeof(Cx<double>) * (size_t)nvec * (m + 1) * mdot_chunks(n)) +
         3 * align_up(sizeof(Cx<double>) * (size_t)nvec * (m + 2)) + align_up(sizeof(double) * nvec) +
         align_up(sizeof(int) * nvec);
}

struct GmresHost {
  std::vector<Cx<double>> R, cs, sn, g;  // R: (m + 1) x m upper part (column j at j * (m + 1)); rotations; rhs
  int len = 0;                            // inner iterations of the current cycle
  bool inner = false;                     // still iterating in this cycle
};

inline Cx<double> cconj(Cx<double> a) { return {a.re, -a.im}; }
inline double cabs2(Cx<double> a) { return a.re * a.re + a.im * a.im; }

template <typename T>
int gmres_impl(lsop_op* op, lsop_precond* pc, const Cx<T>* rhs, Cx<T>* psi, int nvec, double tol, int m, int max_iter,
               int init, const std::vector<int>& start, lsop_solve_info* info, char* ws, hipStream_t s) {
  const size_t n = op->n();
  const size_t vb = align_up(sizeof(Cx<T>) * n * nvec);
  char* w = ws;
  Cx<T>* V = reinterpret_cast<Cx<T>*>(w);
  const size_t bstride = vb / sizeof(Cx<T>);
  w += (size_t)(m + 1) * vb;
  Cx<T>* Zb = reinterpret_cast<Cx<T>*>(w);
  w += vb;
  Cx<T>* Wb = reinterpret_cast<Cx<T>*>(w);
  w += vb;
  Cx<double>* part = reinterpret_cast<Cx<double>*>(w);
  w += align_up(sizeof(Cx<double>) * (size_t)nvec * (m + 1) * mdot_chunks(n));
  const size_t cb = align_up(sizeof(Cx<double>) * (size_t)nvec * (m + 2));
  Cx<double>* h1 = reinterpret_cast<Cx<double>*>(w);
  Cx<double>* h2 = reinterpret_cast<Cx<double>*>(w + cb);
  Cx<double>* coef = reinterpret_cast<Cx<double>*>(w + 2 * cb);
  w += 3 * cb;
  double* dn = reinterpret_cast<double*>(w);
  w += align_up(sizeof(double) * nvec);
  int* dv = reinterpret_cast<int*>(w);
  const int hs = m + 2;  // coefficient column stride

  std::vector<int> act = start;
  if (act.empty())
    for (int v = 0; v < nvec; ++v) act.push_back(v);
  const int na0 = (int)act.size();
  std::vector<double> b2(nvec, 0.0), rn(nvec, 0.0);
  LSOP_HIP(hipMemcpyAsync(dv, act.data(), sizeof(int) * na0, hipMemcpyHostToDevice, s));
  LSOP_HIP(launch_norm2<T>(rhs, dn, dv, na0, n, s));
  LSOP_HIP(hipMemcpyAsync(rn.data(), dn, sizeof(double) * na0, hipMemcpyDeviceToHost, s));
  LSOP_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < na0; ++k) b2[act[k]] = rn[k];
  // start
  if (init == LSOP_INIT_H_RHS) {
    if (pc) {
      int st = pc_apply_impl<T>(pc, rhs, psi, dv, na0, false, s);
      if (st) return st;
    } else {
      LSOP_HIP(launch_axpby<T>(rhs, psi, 1.0, 0.0, dv, na0, n, s));
    }
  } else if (init == LSOP_INIT_ZERO) {
    LSOP_HIP(launch_axpby<T>(rhs, psi, 0.0, 0.0, dv, na0, n, s));
  }
  std::vector<GmresHost> hst(nvec);
  std::vector<int> total(nvec, 0);
  for (int v : act) {
    info[v].iters = 0;
    info[v].status = LSOP_NOT_CONVERGED;
    info[v].rel_residual = INFINITY;
    hst[v].R.assign((size_t)(m + 1) * m, Cx<double>{0, 0});
    hst[v].cs.assign(m, Cx<double>{0, 0});
    hst[v].sn.assign(m, Cx<double>{0, 0});
    hst[v].g.assign(m + 1, Cx<double>{0, 0});
  }
  std::vector<Cx<double>> hc1((size_t)nvec * hs), hc2((size_t)nvec * hs), yc((size_t)nvec * hs);
  for (int cycle = 0;; ++cycle) {
    // true residual r = A psi - psi0 of every active right-hand side
    int na = (int)act.size();
    LSOP_HIP(hipMemcpyAsync(dv, act.data(), sizeof(int) * na, hipMemcpyHostToDevice, s));
    LSOP_HIP(hipMemsetAsync(dn, 0, sizeof(double) * na, s));
    int st = apply_impl<T>(op, LSOP_MODE_A, psi, Wb, rhs, dn, dv, na, s);
    if (st) return st;
    LSOP_HIP(hipMemcpyAsync(rn.data(), dn, sizeof(double) * na, hipMemcpyDeviceToHost, s));
    LSOP_HIP(hipStreamSynchronize(s));
    std::vector<int> next;
    std::vector<double> beta;
    for (int k = 0; k < na; ++k) {
      const int v = act[k];
      const double rel = b2[v] > 0 ? std::sqrt(rn[k] / b2[v]) : std::sqrt(rn[k]);
      info[v].iters = total[v];
      info[v].rel_residual = rel;
      if (cycle == 0) info[v].rel_residual0 = rel;
      if (!std::isfinite(rel)) info[v].status = LSOP_DIVERGED;
      else if (rel <= tol) info[v].status = LSOP_OK;
      else if (total[v] >= max_iter) info[v].status = LSOP_NOT_CONVERGED;
      else {
        next.push_back(v);
        beta.push_back(std::sqrt(rn[k]));
      }
    }
    // v_0 = -r / beta for the right-hand sides that continue (r is still in Wb, slot order of act)
    if (next.empty()) break;
    LSOP_HIP(launch_scale_by_norm<T>(Wb, V, dn, -1.0, dv, na, n, s));  // all of act (finished ones are unused)
    act.swap(next);
    na = (int)act.size();
    for (int k = 0; k < na; ++k) {
      GmresHost& H = hst[act[k]];
      std::fill(H.R.begin(), H.R.end(), Cx<double>{0, 0});
      std::fill(H.g.begin(), H.g.end(), Cx<double>{0, 0});
      H.g[0] = Cx<double>{beta[k], 0.0};
      H.len = 0;
      H.inner = true;
    }
    std::vector<int> in = act;  // right-hand sides still iterating in this cycle
    for (int j = 0; j < m && !in.empty(); ++j) {
      const int ni = (int)in.size();
      LSOP_HIP(hipMemcpyAsync(dv, in.data(), sizeof(int) * ni, hipMemcpyHostToDevice, s));
      Cx<T>* vj = V + (size_t)j * bstride;
      const Cx<T>* src = vj;
      if (pc) {
        if ((st = pc_apply_impl<T>(pc, vj, Zb, dv, ni, false, s))) return st;
        src = Zb;
      }
      if ((st = apply_impl<T>(op, LSOP_MODE_A, src, Wb, nullptr, nullptr, dv, ni, s))) return st;
      // classical Gram-Schmidt against v_0 .. v_j, twice
      LSOP_HIP(launch_mdot<T>(V, bstride, j + 1, Wb, dv, ni, n, part, h1, hs, false, s));
      LSOP_HIP(launch_mcombine<T>(V, bstride, j + 1, h1, hs, -1.0, 1.0, Wb, dv, ni, n, s));
      LSOP_HIP(launch_mdot<T>(V, bstride, j + 1, Wb, dv, ni, n, part, h2, hs, false, s));
      LSOP_HIP(launch_mcombine<T>(V, bstride, j + 1, h2, hs, -1.0, 1.0, Wb, dv, ni, n, s));
      LSOP_HIP(launch_norm2<T>(Wb, dn, dv, ni, n, s));
      LSOP_HIP(launch_scale_by_norm<T>(Wb, V + (size_t)(j + 1) * bstride, dn, 1.0, dv, ni, n, s));
      LSOP_HIP(hipMemcpyAsync(hc1.data(), h1, sizeof(Cx<double>) * (size_t)ni * hs, hipMemcpyDeviceToHost, s));
      LSOP_HIP(hipMemcpyAsync(hc2.data(), h2, sizeof(Cx<double>) * (size_t)ni * hs, hipMemcpyDeviceToHost, s));
      LSOP_HIP(hipMemcpyAsync(rn.data(), dn, sizeof(double) * ni, hipMemcpyDeviceToHost, s));
      LSOP_HIP(hipStreamSynchronize(s));
      std::vector<int> keep;
      for (int k = 0; k < ni; ++k) {
        const int v = in[k];
        GmresHost& H = hst[v];
        Cx<double>* col = H.R.data() + (size_t)j * (m + 1);
        for (int i = 0; i <= j; ++i) {
          const Cx<double> a = hc1[(size_t)k * hs + i], b = hc2[(size_t)k * hs + i];
          col[i] = Cx<double>{a.re + b.re, a.im + b.im};
        }
        const double hn = std::sqrt(rn[k]);
        col[j + 1] = Cx<double>{hn, 0.0};
        // earlier rotations, then a new one that zeroes col[j + 1]
        for (int i = 0; i < j; ++i) {
          const Cx<double> x = col[i], y = col[i + 1];
          const double c = H.cs[i].re;
          const Cx<double> sv = H.sn[i];
          col[i] = Cx<double>{c * x.re + sv.re * y.re - sv.im * y.im, c * x.im + sv.re * y.im + sv.im * y.re};
          const Cx<double> sc = cconj(sv);
          col[i + 1] = Cx<double>{-(sc.re * x.re - sc.im * x.im) + c * y.re, -(sc.re * x.im + sc.im * x.re) + c * y.im};
        }
        const Cx<double> a = col[j], b = col[j + 1];
        const double na_ = std::sqrt(cabs2(a)), t = std::sqrt(cabs2(a) + cabs2(b));
        double c = 1.0;
        Cx<double> sv{0.0, 0.0};
        if (t > 0.0) {
          if (na_ == 0.0) {
            c = 0.0;
            sv = Cx<double>{cconj(b).re / t, cconj(b).im / t};
            col[j] = Cx<double>{t, 0.0};
          } else {
            c = na_ / t;
            const Cx<double> ph{a.re / na_, a.im / na_};
            const Cx<double> cb = cconj(b);
            sv = Cx<double>{(ph.re * cb.re - ph.im * cb.im) / t, (ph.re * cb.im + ph.im * cb.re) / t};
            col[j] = Cx<double>{ph.re * t, ph.im * t};
          }
        }
        col[j + 1] = Cx<double>{0.0, 0.0};
        H.cs[j] = Cx<double>{c, 0.0};
        H.sn[j] = sv;
        const Cx<double> gj = H.g[j];
        const Cx<double> sc = cconj(sv);
        H.g[j + 1] = Cx<double>{-(sc.re * gj.re - sc.im * gj.im), -(sc.re * gj.im + sc.im * gj.re)};
        H.g[j] = Cx<double>{c * gj.re, c * gj.im};
        H.len = j + 1;
        ++total[v];
        const double est = std::sqrt(cabs2(H.g[j + 1]));
        const double bnorm = b2[v] > 0 ? std::sqrt(b2[v]) : 1.0;
        if (!(est / bnorm > tol) || hn == 0.0 || total[v] >= max_iter || !std::isfinite(est)) continue;
        keep.push_back(v);
      }
      in.swap(keep);
    }
    // psi += H (V y) with R y = g for each right-hand side of the cycle
    int maxlen = 0;
    std::fill(yc.begin(), yc.end(), Cx<double>{0, 0});
    for (int k = 0; k < na; ++k) {
      GmresHost& H = hst[act[k]];
      const int L = H.len;
      maxlen = std::max(maxlen, L);
      Cx<double>* y = yc.data() + (size_t)k * hs;
      for (int i = L - 1; i >= 0; --i) {
        Cx<double> acc = H.g[i];
        for (int q = i + 1; q < L; ++q) {
          const Cx<double> r = H.R[(size_t)q * (m + 1) + i];
          acc = Cx<double>{acc.re - (r.re * y[q].re - r.im * y[q].im), acc.im - (r.re * y[q].im + r.im * y[q].re)};
        }
        const Cx<double> d = H.R[(size_t)i * (m + 1) + i];
        const double dd = cabs2(d);
        y[i] = dd > 0.0 ? Cx<double>{(acc.re * d.re + acc.im * d.im) / dd, (acc.im * d.re - acc.re * d.im) / dd}
                        : Cx<double>{0.0, 0.0};
      }
    }
    LSOP_HIP(hipMemcpyAsync(dv, act.data(), sizeof(int) * na, hipMemcpyHostToDevice, s));
    LSOP_HIP(hipMemcpyAsync(coef, yc.data(), sizeof(Cx<double>) * (size_t)na * hs, hipMemcpyHostToDevice, s));
    LSOP_HIP(launch_mcombine<T>(V, bstride, maxlen, coef, hs, 1.0, 0.0, Zb, dv, na, n, s));
    const Cx<T>* upd = Zb;
    if (pc) {
      if ((st = pc_apply_impl<T>(pc, Zb, Wb, dv, na, false, s))) return st;
      upd = Wb;
    }
    LSOP_HIP(launch_axpby<T>(upd, psi, 1.0, 1.0, dv, na, n, s));
  }
  return LSOP_OK;
}

// Iterative refinement of a complex-FP64 solve (LSOP_MIXED): outer FP64 residuals r = A psi - psi0 and the
// accumulated psi in FP64, inner solves of A d = r in complex FP32 (any inner method), psi <- psi - d, until
// the FP64 relative residual <= tol.  Workspace at base: r (FP64), r and d (FP32), norms, active list
// (refine_ws_bytes); the inner method's own workspace follows it.
size_t refine_ws_bytes(size_t n, int nvec) {
  return align_up(sizeof(Cx<double>) * n * nvec) + 2 * align_up(sizeof(Cx<float>) * n * nvec) +
         align_up(sizeof(double) * nvec) + align_up(sizeof(int) * nvec);
}

int overall_status(const lsop_solve_info* info, int nvec);

template <typename Inner>
int refine_impl(lsop_op* op, const Cx<double>* rhs, Cx<double>* psi, int nvec, double tol, int refine_max, int init,
                lsop_solve_info* info, char* base, hipStream_t s, Inner&& inner) {
  const size_t n = op->n();
  const size_t b64 = align_up(sizeof(Cx<double>) * n * nvec), b32 = align_up(sizeof(Cx<float>) * n * nvec);
  Cx<double>* r64 = (Cx<double>*)base;
  Cx<float>* rhs32 = (Cx<float>*)(base + b64);
  Cx<float>* d32 = (Cx<float>*)(base + b64 + b32);
  double* dn = (double*)(base + b64 + 2 * b32);
  int* dv = (int*)((char*)dn + align_up(sizeof(double) * nvec));
  std::vector<int> active(nvec);
  for (int v = 0; v < nvec; ++v) active[v] = v;
  std::vector<double> b2(nvec), rn(nvec);
  LSOP_HIP(hipMemcpyAsync(dv, active.data(), sizeof(int) * nvec, hipMemcpyHostToDevice, s));
  LSOP_HIP(launch_norm2<double>(rhs, dn, dv, nvec, n, s));
  LSOP_HIP(hipMemcpyAsync(b2.data(), dn, sizeof(double) * nvec, hipMemcpyDeviceToHost, s));
  LSOP_HIP(hipStreamSynchronize(s));
  if (init != LSOP_INIT_USER && init != LSOP_INIT_BEST)
    LSOP_HIP(hipMemsetAsync(psi, 0, sizeof(Cx<double>) * n * nvec, s));
  std::vector<lsop_solve_info> inn(nvec);
  std::vector<int> total_iters(nvec, 0);
  int st = 0;
  for (int k = 0;; ++k) {
    const int na = (int)active.size();
    LSOP_HIP(hipMemcpyAsync(dv, active.data(), sizeof(int) * na, hipMemcpyHostToDevice, s));
    LSOP_HIP(hipMemsetAsync(dn, 0, sizeof(double) * na, s));
    // FP64 residual r = A psi - psi0
    if ((st = apply_impl<double>(op, LSOP_MODE_A, psi, r64, rhs, dn, dv, na, s))) return st;
    LSOP_HIP(hipMemcpyAsync(rn.data(), dn, sizeof(double) * na, hipMemcpyDeviceToHost, s));
    LSOP_HIP(hipStreamSynchronize(s));
    std::vector<int> next;
    for (int j = 0; j < na; ++j) {
      const int v = active[j];
      const double rel = b2[v] > 0 ? std::sqrt(rn[j] / b2[v]) : std::sqrt(rn[j]);
      info[v].rel_residual = rel;
      if (k == 0) info[v].rel_residual0 = rel;
      info[v].refine_steps = k;
      info[v].iters = total_iters[v];
      if (!std::isfinite(rel)) info[v].status = LSOP_DIVERGED;
      else if (rel <= tol) info[v].status = LSOP_OK;
      else if (k == refine_max) info[v].status = LSOP_NOT_CONVERGED;
      else if (k > 0 && inn[v].status == LSOP_DIVERGED) info[v].status = LSOP_DIVERGED;
      else next.push_back(v);
    }
    active.swap(next);
    if (active.empty()) break;
    // inner FP32 solve of A d = r; psi <- psi - d
    LSOP_HIP(launch_convert<float, double>(r64, rhs32, n * nvec, s));
    if ((st = inner(rhs32, d32, active, inn.data(), dn, dv))) return st;
    const int nn = (int)active.size();
    LSOP_HIP(hipMemcpyAsync(dv, active.data(), sizeof(int) * nn, hipMemcpyHostToDevice, s));
    LSOP_HIP(launch_accumulate<float>(d32, psi, -1.0, dv, nn, n, s));
    for (int v : active) total_iters[v] += inn[v].iters;
  }
  return overall_status(info, nvec);
}

int overall_status(const lsop_solve_info* info, int nvec) {
  for (int v = 0; v < nvec; ++v)
    if (info[v].status != LSOP_OK) return info[v].status;
  return LSOP_OK;
}


// ------------------------------------------------------------------ batches
// Several operators (instances of possibly different sizes, each with its own
// contrast and spectrum) advanced together: instances of the same grid shape
// form a group, and every FFT pass is one launch per group whose slots (one
// per vector) carry their own operands.

int grow_buf(void** p, size_t* cap, size_t need, size_t* bytes) {
  if (need <= *cap) return LSOP_OK;
  if (*p) {
    LSOP_HIP(hipDeviceSynchronize());
    (void)hipFree(*p);
    *bytes -= *cap;
    *p = nullptr;
    *cap = 0;
  }
  if (lib_malloc(p, need) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LSOP_ENOMEM, "batch allocation of " + std::to_string(need) + " bytes failed");
  }
  *cap = need;
  *bytes += need;
  return LSOP_OK;
}

// Host slot tables of all groups (group by group, member by member, vector by
// vector); goff[g] = first slot of group g.  slot_of[i] = first slot of instance i.
template <typename T>
void batch_slots(lsop_batch* b, const Cx<T>* const* x, Cx<T>* const* y, const Cx<T>* const* rhs, double* rnorm,
                 const int* nvec, std::vector<int>& goff, std::vector<int>& slot_of) {
  goff.assign(b->groups.size() + 1, 0);
  slot_of.assign(b->count, 0);
  std::vector<Slot<T>> all;
  for (size_t g = 0; g < b->groups.size(); ++g) {
    goff[g] = (int)all.size();
    for (int i : b->groups[g].members) {
      lsop_op* op = b->ops[i];
      const size_t n = op->n();
      slot_of[i] = (int)all.size();
      for (int v = 0; v < nvec[i]; ++v) {
        Slot<T> sl;
        sl.x = x[i] + (size_t)v * n;
        sl.y = y[i] + (size_t)v * n;
        sl.rhs = rhs ? rhs[i] + (size_t)v * n : nullptr;
        sl.chi = Dt<T>::chi(op);
        sl.gs = Dt<T>::gs(op);
        sl.rnorm = rnorm ? rnorm + all.size() : nullptr;
        all.push_back(sl);
      }
    }
  }
  goff[b->groups.size()] = (int)all.size();
  b->host_tab.resize(all.size() * sizeof(Slot<T>));
  if (!all.empty()) memcpy(b->host_tab.data(), all.data(), b->host_tab.size());
}

// upload the host tables and size the grouped intermediate
template <typename T>
int batch_prepare(lsop_batch* b, const std::vector<int>& goff, hipStream_t s) {
  int st = grow_buf(&b->tab, &b->tab_cap, std::max<size_t>(b->host_tab.size(), 16), &b->bytes);
  if (st) return st;
  size_t tneed = 16;
  for (size_t g = 0; g < b->groups.size(); ++g) {
    const auto& G = b->groups[g];
    tneed = std::max(tneed, sizeof(Cx<T>) * (size_t)(goff[g + 1] - goff[g]) * G.nx * 2 * G.lz);
  }
  if ((st = grow_buf(&b->tmp, &b->tmp_cap, tneed, &b->bytes))) return st;
  if (!b->host_tab.empty()) {
    LSOP_HIP(hipMemcpyAsync(b->tab, b->host_tab.data(), b->host_tab.size(), hipMemcpyHostToDevice, s));
    LSOP_HIP(hipStreamSynchronize(s));  // the staging buffer is reused by the next call
  }
  return LSOP_OK;
}

// The three passes of `mode` for every group, one launch per pass per group.
template <typename T>
int batch_passes(lsop_batch* b, int mode, const std::vector<int>& goff, bool residual, hipStream_t s) {
  const Slot<T>* tab = reinterpret_cast<const Slot<T>*>(b->tab);
  Cx<T>* tmp = reinterpret_cast<Cx<T>*>(b->tmp);
  const bool mulchi = (mode == LSOP_MODE_A || mode == LSOP_MODE_G0V), adj = !mulchi;
  const bool xin = (mode == LSOP_MODE_A || mode == LSOP_MODE_AH);
  const bool chi_out = (mode == LSOP_MODE_AH || mode == LSOP_MODE_VHG0H);
  for (size_t g = 0; g < b->groups.size(); ++g) {
    const auto& G = b->groups[g];
    const int ns = goff[g + 1] - goff[g];
    if (ns == 0) continue;
    lsop_op* op0 = b->ops[G.members[0]];
    const Slot<T>* tg = tab + goff[g];
    const double e = sizeof(Cx<T>), t = sizeof(T), nn = (double)op0->n(), np = (double)op0->nx * op0->pz();
    std::string fcol;
    LSOP_HIP(prof("batch_rows_fwd", fn_name("k_rows_fwd", tname<T>(), G.lz), ns * (nn * e + np * e + (mulchi ? nn * t : 0.0)),
                  0.0, ns, s, [&] {
                    return launch_rows_fwd<T>(G.lz, nullptr, nullptr, tmp, nullptr, G.nx, G.nz, ns, mulchi,
                                              Dt<T>::twz(op0), s, 1, 0, -1, tg);
                  }));
    LSOP_HIP(prof("batch_cols", fcol, ns * (2.0 * np * e + 2.0 * op0->pz() * G.lx * e), 0.0, ns, s, [&] {
      int used = 0;
      hipError_t er = launch_cols<T>(G.lx, tmp, nullptr, G.nx, op0->pz(), ns, adj, Dt<T>::twx(op0), s, G.col_tile,
                                     &used, tg);
      fcol = fn_name("k_cols", tname<T>(), G.lx, used);
      return er;
    }));
    LSOP_HIP(prof("batch_rows_inv", fn_name("k_rows_inv", tname<T>(), G.lz),
                  ns * (np * e + nn * e + (xin ? nn * e : 0.0) + (residual ? nn * e : 0.0) + (chi_out ? nn * t : 0.0)),
                  0.0, ns, s, [&] {
                    return launch_rows_inv<T>(G.lz, tmp, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, G.nx,
                                              G.nz, ns, mode, Dt<T>::twz(op0), s, 1, 0, -1, tg);
                  }));
  }
  return LSOP_OK;
}

template <typename T>
int batch_apply_impl(lsop_batch* b, int mode, const Cx<T>* const* x, Cx<T>* const* y, const int* nvec, hipStream_t s) {
  std::vector<int> goff, slot_of;
  batch_slots<T>(b, x, y, nullptr, nullptr, nvec, goff, slot_of);
  int st = batch_prepare<T>(b, goff, s);
  if (st) return st;
  return batch_passes<T>(b, mode, goff, false, s);
}

// One iteration of the grouped series (after the residuals of the previous
// one): freeze finished vectors (zero their residual), psi <- psi - H r for
// every instance, then r = A psi - rhs with |r|^2 per slot.
template <typename T>
int batch_iteration(lsop_batch* b, lsop_precond* const* pcs, Cx<T>* const* psi, Cx<T>* const* r, const int* nvec,
                    const std::vector<int>& goff, double* rn, const int* live, int nslots, hipStream_t s) {
  const Slot<T>* tab = reinterpret_cast<const Slot<T>*>(b->tab);
  for (size_t g = 0; g < b->groups.size(); ++g) {
    const int ns = goff[g + 1] - goff[g];
    const auto& G = b->groups[g];
    LSOP_HIP(launch_mask_slots<T>(tab + goff[g], live + goff[g], ns, (size_t)G.nx * G.nz, s));
  }
  // psi_i <- psi_i - H_i r_i: independent per instance (each preconditioner has its own scratch), so the
  // instances are spread over the side streams, which fork from and join back into s (also under capture,
  // where they become parallel branches of the graph)
  const int K = b->active_side;
  if (K > 0) {
    LSOP_HIP(hipEventRecord(b->ev[0], s));
    for (int k = 0; k < K; ++k) LSOP_HIP(hipStreamWaitEvent(b->side[k], b->ev[0], 0));
  }
  int j = 0;
  for (int i = 0; i < b->count; ++i) {
    if (nvec[i] == 0) continue;
    hipStream_t si = K > 0 ? b->side[j++ % K] : s;
    if (pcs && pcs[i] && pcs[i]->kind != LSOP_PC_IDENTITY) {
      int st = pc_apply_impl<T>(pcs[i], r[i], psi[i], nullptr, nvec[i], true, si);
      if (st) return st;
    } else {
      LSOP_HIP(launch_axpby<T>(r[i], psi[i], -1.0, 1.0, nullptr, nvec[i], b->ops[i]->n(), si));
    }
  }
  for (int k = 0; k < K; ++k) {
    LSOP_HIP(hipEventRecord(b->ev[1 + k], b->side[k]));
    LSOP_HIP(hipStreamWaitEvent(s, b->ev[1 + k], 0));
  }
  LSOP_HIP(launch_zero_f64(rn, nslots, s));
  return batch_passes<T>(b, LSOP_MODE_A, goff, true, s);
}

// Side streams for the per-instance applies of the series: up to kSeriesStreams, none when fewer than two
// instances apply a preconditioner or when one preconditioner serves two instances (their applies would
// share its scratch).
constexpr int kSeriesStreams = 8;
int batch_side_streams(lsop_batch* b, lsop_precond* const* pcs, const int* nvec) {
  int busy = 0;
  bool shared = false;
  std::vector<const lsop_precond*> seen;
  for (int i = 0; i < b->count; ++i) {
    if (nvec[i] == 0) continue;
    ++busy;
    if (pcs && pcs[i] && pcs[i]->kind != LSOP_PC_IDENTITY) {
      shared = shared || std::find(seen.begin(), seen.end(), pcs[i]) != seen.end();
      seen.push_back(pcs[i]);
    }
  }
  const int want = (!shared && busy >= 2) ? std::min(busy, kSeriesStreams) : 0;
  while ((int)b->side.size() < want) {
    hipStream_t st = nullptr;
    LSOP_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    b->side.push_back(st);
  }
  while ((int)b->ev.size() < 1 + (int)b->side.size()) {
    hipEvent_t e = nullptr;
    LSOP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->ev.push_back(e);
  }
  b->active_side = want;  // streams created for an earlier, larger series stay for later calls
  return LSOP_OK;
}

template <typename T>
int batch_series(lsop_batch* b, lsop_precond* const* pcs, const Cx<T>* const* rhs, Cx<T>* const* psi, const int* nvec,
                 const lsop_solve_params* p, bool use_graph, lsop_solve_info* info, hipStream_t user_s) {
  const int cnt = b->count;
  // work: residual vectors, norms, live flags
  std::vector<size_t> roff(cnt);
  size_t rtot = 0;
  int nslots = 0;
  for (int i = 0; i < cnt; ++i) {
    roff[i] = rtot;
    rtot += (size_t)nvec[i] * b->ops[i]->n();
    nslots += nvec[i];
  }
  if (nslots == 0) return LSOP_OK;
  const size_t rb = align_up(sizeof(Cx<T>) * rtot), nb = align_up(sizeof(double) * nslots);
  int st = grow_buf(&b->work, &b->work_cap, rb + nb + align_up(sizeof(int) * nslots), &b->bytes);
  if (st) return st;
  Cx<T>* rbase = reinterpret_cast<Cx<T>*>(b->work);
  double* rn = reinterpret_cast<double*>((char*)b->work + rb);
  int* live = reinterpret_cast<int*>((char*)b->work + rb + nb);
  std::vector<Cx<T>*> r(cnt);
  for (int i = 0; i < cnt; ++i) r[i] = rbase + roff[i];
  // captured work runs on a stream of its own (the legacy default stream cannot be captured)
  hipStream_t s = user_s;
  hipStream_t own = nullptr;
  if (use_graph) {
    LSOP_HIP(hipStreamSynchronize(user_s));
    LSOP_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
    s = own;
  }
  struct Cleanup {
    hipStream_t st = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~Cleanup() {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
      }
    }
  } cl;
  cl.st = own;
  std::vector<int> goff, slot_of;
  batch_slots<T>(b, reinterpret_cast<const Cx<T>* const*>(psi), r.data(), rhs, rn, nvec, goff, slot_of);
  if ((st = batch_prepare<T>(b, goff, s))) return st;
  if ((st = batch_side_streams(b, pcs, nvec))) return st;
  // |rhs|^2 per slot and psi_0
  std::vector<double> b2(nslots), rh(nslots);
  std::vector<int> liveh(nslots, 1), rising(nslots, 0), done(nslots, 0);
  std::vector<double> prev(nslots, INFINITY);
  // psi_0 = H rhs per instance, spread over the side streams as in the iterations
  const int K = b->active_side;
  if (K > 0) {
    LSOP_HIP(hipEventRecord(b->ev[0], s));
    for (int k = 0; k < K; ++k) LSOP_HIP(hipStreamWaitEvent(b->side[k], b->ev[0], 0));
  }
  for (int i = 0, j = 0; i < cnt; ++i) {
    if (nvec[i] == 0) continue;
    const size_t n = b->ops[i]->n();
    hipStream_t si = K > 0 ? b->side[j++ % K] : s;
    LSOP_HIP(launch_norm2<T>(rhs[i], rn + slot_of[i], nullptr, nvec[i], n, si));
    if (p->init == LSOP_INIT_H_RHS) {
      if (pcs && pcs[i] && pcs[i]->kind != LSOP_PC_IDENTITY) {
        if ((st = pc_apply_impl<T>(pcs[i], rhs[i], psi[i], nullptr, nvec[i], false, si))) return st;
      } else {
        LSOP_HIP(launch_axpby<T>(rhs[i], psi[i], 1.0, 0.0, nullptr, nvec[i], n, si));
      }
    } else if (p->init == LSOP_INIT_ZERO) {
      LSOP_HIP(launch_axpby<T>(rhs[i], psi[i], 0.0, 0.0, nullptr, nvec[i], n, si));
    }
  }
  for (int k = 0; k < K; ++k) {
    LSOP_HIP(hipEventRecord(b->ev[1 + k], b->side[k]));
    LSOP_HIP(hipStreamWaitEvent(s, b->ev[1 + k], 0));
  }
  LSOP_HIP(hipMemcpyAsync(b2.data(), rn, sizeof(double) * nslots, hipMemcpyDeviceToHost, s));
  LSOP_HIP(hipStreamSynchronize(s));
  // slot -> (instance, vector) for the per-vector report (info is in instance order)
  std::vector<int> info_of(nslots);
  {
    std::vector<int> ibase(cnt, 0);
    int acc = 0;
    for (int i = 0; i < cnt; ++i) {
      ibase[i] = acc;
      acc += nvec[i];
    }
    for (int i = 0; i < cnt; ++i)
      for (int v = 0; v < nvec[i]; ++v) info_of[slot_of[i] + v] = ibase[i] + v;
  }
  LSOP_HIP(launch_zero_f64(rn, nslots, s));
  if ((st = batch_passes<T>(b, LSOP_MODE_A, goff, true, s))) return st;
  const bool prof_was = g_prof;
  for (int it = 0;; ++it) {
    LSOP_HIP(hipMemcpyAsync(rh.data(), rn, sizeof(double) * nslots, hipMemcpyDeviceToHost, s));
    LSOP_HIP(hipStreamSynchronize(s));
    int nlive = 0;
    for (int k = 0; k < nslots; ++k) {
      if (done[k]) continue;
      lsop_solve_info& in = info[info_of[k]];
      const double rel = b2[k] > 0 ? std::sqrt(rh[k] / b2[k]) : std::sqrt(rh[k]);
      in.iters = it;
      in.rel_residual = rel;
      if (it == 0) in.rel_residual0 = rel;
      int stt = -1;
      if (!std::isfinite(rel)) stt = LSOP_DIVERGED;
      else if (rel <= p->tol) stt = LSOP_OK;
      else {
        rising[k] = rel > prev[k] ? rising[k] + 1 : 0;
        prev[k] = rel;
        if (rising[k] >= 5) stt = LSOP_DIVERGED;
        else if (it == p->max_iter) stt = LSOP_NOT_CONVERGED;
      }
      if (stt >= 0) {
        in.status = stt;
        done[k] = 1;
        liveh[k] = 0;
      } else {
        ++nlive;
      }
    }
    if (nlive == 0) break;
    LSOP_HIP(hipMemcpyAsync(live, liveh.data(), sizeof(int) * nslots, hipMemcpyHostToDevice, s));
    if (!use_graph) {
      if ((st = batch_iteration<T>(b, pcs, psi, r.data(), nvec, goff, rn, live, nslots, s))) return st;
      continue;
    }
    if (!cl.exec) {
      LSOP_HIP(hipStreamSynchronize(s));  // the live flags are in place before capture starts
      g_prof = false;
      LSOP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
      st = batch_iteration<T>(b, pcs, psi, r.data(), nvec, goff, rn, live, nslots, s);
      const hipError_t ec = hipStreamEndCapture(s, &cl.graph);
      g_prof = prof_was;
      if (st) return st;
      LSOP_HIP(ec);
      LSOP_HIP(hipGraphInstantiate(&cl.exec, cl.graph, nullptr, nullptr, 0));
    }
    LSOP_HIP(hipGraphLaunch(cl.exec, s));
  }
  return LSOP_OK;
}

}  // namespace

hipError_t prof_launch(const char* name, const char* fn, double bytes, double flops, double items, hipStream_t s,
                       const std::function<hipError_t()>& launch) {
  return prof(name, fn, bytes, flops, items, s, launch);
}

size_t apply_tmp_bytes_per_vec(const lsop_op* op) {
  return (op->has64() ? sizeof(Cx<double>) : sizeof(Cx<float>)) * (size_t)op->nx * op->py() * op->pz();
}

int apply_into(lsop_op* op, int mode, const void* x, void* y, int nvec, void* tmp, int chunk, hipStream_t s) {
  int st = check_op(op);
  if (st) return st;
  if (mode < 0 || mode > 3) return fail(LSOP_EINVAL, "bad mode");
  if (nvec < 0 || (nvec > 0 && (!x || !y))) return fail(LSOP_EINVAL, "bad vectors");
  if (nvec == 0) return LSOP_OK;
  if (op->dtype == LSOP_C64)
    return apply_impl<float>(op, mode, (const Cx<float>*)x, (Cx<float>*)y, nullptr, nullptr, nullptr, nvec, s, tmp,
                             chunk);
  return apply_impl<double>(op, mode, (const Cx<double>*)x, (Cx<double>*)y, nullptr, nullptr, nullptr, nvec, s, tmp,
                            chunk);
}
}  // namespace lsop

using namespace lsop;

extern "C" {

const char* lsop_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace lsop {
namespace {

// Validates lsop_create's arguments and fills the plan fields of a fresh handle.
int op_plan(int nx, int nz, int dtype, int max_vec, lsop_op* op) {
  if (nx < 1 || nz < 1 || max_vec < 1) return fail(LSOP_EINVAL, "nx, nz and max_vec must be >= 1");
  if (dtype != LSOP_C64 && dtype != LSOP_C128 && dtype != LSOP_MIXED) return fail(LSOP_EUNSUPPORTED, "bad dtype");
  const int lx = fft_length_for(nx), lz = fft_length_for(nz);
  if (lx < 0 || lz < 0) return fail(LSOP_EUNSUPPORTED, "grid side exceeds the largest FFT length (2048)");
  if ((size_t)nx * nz > (size_t)INT32_MAX / 2) return fail(LSOP_EUNSUPPORTED, "grid too large");
  op->nx = nx;
  op->nz = nz;
  op->lx = lx;
  op->lz = lz;
  op->dtype = dtype;
  op->max_vec = max_vec;
  op->src_cap = 4096;
  if (const char* ct = getenv("LSOP_COL_TILE")) op->col_tile = atoi(ct);
  return LSOP_OK;
}

// Every device buffer of an operator's state, in one fixed order (the size query walks the same list).
int op_buffers(lsop_op* op, Alloc& a) {
  const size_t n = op->n();
  const size_t px = op->px(), pz = op->pz();
  const int lx = op->lx, lz = op->lz;
  int st = 0;
  const size_t py = op->py();
  st |= dev_alloc(a, &op->chi64, sizeof(double) * n);
  if (op->has32()) st |= dev_alloc(a, &op->chi32, sizeof(float) * n);
  st |= dev_alloc(a, &op->ktab, sizeof(Cx<double>) * n);
  if (op->has64()) st |= dev_alloc(a, &op->gs64, sizeof(Cx<double>) * px * py * pz);
  if (op->has32()) st |= dev_alloc(a, &op->gs32, sizeof(Cx<float>) * px * py * pz);
  st |= dev_alloc(a, &op->tw2x64, sizeof(Cx<double>) * 2 * lx);
  st |= dev_alloc(a, &op->tw2z64, sizeof(Cx<double>) * 2 * lz);
  if (op->dims == 3) st |= dev_alloc(a, &op->tw2y64, sizeof(Cx<double>) * 2 * op->ly);
  if (op->has32()) {
    st |= dev_alloc(a, &op->tw2x32, sizeof(Cx<float>) * 2 * lx);
    st |= dev_alloc(a, &op->tw2z32, sizeof(Cx<float>) * 2 * lz);
    if (op->dims == 3) st |= dev_alloc(a, &op->tw2y32, sizeof(Cx<float>) * 2 * op->ly);
  }
  const size_t esz = op->has64() ? sizeof(Cx<double>) : sizeof(Cx<float>);
  st |= dev_alloc(a, &op->tmp, esz * (size_t)op->max_vec * op->nx * py * pz);
  st |= dev_alloc(a, &op->flag, 256);
  st |= dev_alloc(a, &op->dsrc, sizeof(int) * 3 * op->src_cap);
  st |= dev_alloc(a, &op->damp, sizeof(Cx<double>) * op->src_cap);
  return st ? LSOP_ENOMEM : LSOP_OK;
}

// Twiddle tables of both axes (host-computed, uploaded synchronously).
int op_twiddles(lsop_op* op) {
  for (int axis = 0; axis < op->dims; ++axis) {
    const int L = axis == 0 ? op->lx : axis == 1 ? op->lz : op->ly;
    std::vector<Cx<double>> w = twiddles(L);
    Cx<double>* d64 = axis == 0 ? op->tw2x64 : axis == 1 ? op->tw2z64 : op->tw2y64;
    if (hipMemcpy(d64, w.data(), sizeof(Cx<double>) * w.size(), hipMemcpyHostToDevice) != hipSuccess)
      return fail(LSOP_EHIP, "twiddle upload failed");
    if (op->has32()) {
      std::vector<Cx<float>> w32(w.size());
      for (size_t t = 0; t < w.size(); ++t) w32[t] = ccast<float>(w[t]);
      Cx<float>* d32 = axis == 0 ? op->tw2x32 : axis == 1 ? op->tw2z32 : op->tw2y32;
      if (hipMemcpy(d32, w32.data(), sizeof(Cx<float>) * w32.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail(LSOP_EHIP, "twiddle upload failed");
    }
  }
  return LSOP_OK;
}

// 3D plan on top of the 2D one: the y axis, its FFT length, and the size limit of the flattened index.
int op_plan3(int nx, int ny, int nz, int dtype, int max_vec, lsop_op* op) {
  int st = op_plan(nx, nz, dtype, max_vec, op);
  if (st) return st;
  if (ny < 1) return fail(LSOP_EINVAL, "ny must be >= 1");
  const int ly = fft_length_for(ny);
  if (ly < 0) return fail(LSOP_EUNSUPPORTED, "grid side exceeds the largest FFT length (2048)");
  if ((size_t)nx * ny * nz > (size_t)INT32_MAX / 4 || (size_t)nx * 2 * ly * 2 * op->lz > (size_t)INT32_MAX)
    return fail(LSOP_EUNSUPPORTED, "3D grid too large");
  op->ny = ny;
  op->ly = ly;
  op->dims = 3;
  return LSOP_OK;
}

int op_create(int nx, int nz, int dtype, int max_vec, void* state, size_t state_bytes, lsop_op** out, int ny = 0) {
  if (!out) return fail(LSOP_EINVAL, "null output handle");
  *out = nullptr;
  lsop_op* op = new lsop_op();
  int st = ny > 0 ? op_plan3(nx, ny, nz, dtype, max_vec, op) : op_plan(nx, nz, dtype, max_vec, op);
  if (st) {
    delete op;
    return st;
  }
  Alloc a;
  a.owned = &op->owned;
  a.bytes = &op->bytes;
  if (state) {
    a.base = reinterpret_cast<char*>(state);
    a.cap = state_bytes;
    op->state_external = true;
  }
  if ((st = op_buffers(op, a)) || (st = op_twiddles(op))) {
    free_all(op->owned);
    delete op;
    return st;
  }
  *out = op;
  return LSOP_OK;
}

}  // namespace
}  // namespace lsop

extern "C" {

int lsop_create(int nx, int nz, int dtype, int max_vec, lsop_op** out) {
  return op_create(nx, nz, dtype, max_vec, nullptr, 0, out);
}

int lsop_create_in(int nx, int nz, int dtype, int max_vec, void* state_dev, size_t state_bytes, lsop_op** out) {
  if (!state_dev || (reinterpret_cast<uintptr_t>(state_dev) & 255) != 0)
    return fail(LSOP_EINVAL, "state buffer must be non-null and 256-byte aligned");
  return op_create(nx, nz, dtype, max_vec, state_dev, state_bytes, out);
}

int lsop_state_bytes(int nx, int nz, int dtype, int max_vec, size_t* bytes) {
  if (!bytes) return fail(LSOP_EINVAL, "null output");
  lsop_op op;
  int st = op_plan(nx, nz, dtype, max_vec, &op);
  if (st) return st;
  size_t total = 0;
  Alloc a;
  a.bytes = &total;
  a.count_only = true;
  (void)op_buffers(&op, a);
  *bytes = total;
  return LSOP_OK;
}

int lsop_set_problem(lsop_op* op, const double* vel_dev, double h, double freq_hz, double c0, void* stream) {
  if (!op) return fail(LSOP_EINVAL, "null operator handle");
  if (op->dims == 3) return fail(LSOP_EINVAL, "3D operator: use lsop_set_problem3d");
  if (!vel_dev) return fail(LSOP_EINVAL, "null velocity");
  if (!(h > 0) || !(freq_hz > 0) || !(c0 > 0) || !std::isfinite(h) || !std::isfinite(freq_hz) || !std::isfinite(c0))
    return fail(LSOP_EINVAL, "h, freq_hz and c0 must be positive and finite");
  const double pi = lsop_bessel::kPi;
  const double w = 2.0 * pi * freq_hz;
  const double k0 = w / c0;
  const double a = h / std::sqrt(pi);
  const double ka = k0 * a;
  if (ka > 2.0) return fail(LSOP_EINVAL, "grid too coarse: k0 h / sqrt(pi) > 2");
  hipStream_t s = S(stream);
  const size_t n = op->n();
  op->damped = false;
  LSOP_HIP(hipMemsetAsync(op->flag, 0, sizeof(unsigned), s));
  LSOP_HIP(launch_contrast(vel_dev, op->chi64, op->chi32, (int)n, w * w, 1.0 / (c0 * c0), op->flag, s));
  unsigned bad = 0;
  LSOP_HIP(hipMemcpyAsync(&bad, op->flag, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  LSOP_HIP(hipStreamSynchronize(s));
  if (bad) {
    op->ready = false;
    return fail(LSOP_EINVAL, "velocity must be finite and positive");
  }
  // self cell and the J1 factor of the disk-integrated kernel
  double j1 = 0, y1 = 0;
  lsop_bessel::bessel1_small(ka, &j1, &y1);
  const Cx<double> c{0.0, pi * a / (2.0 * k0)};
  const Cx<double> cj1 = c * Cx<double>{j1, 0.0};
  const Cx<double> self = c * Cx<double>{j1, y1} - Cx<double>{1.0 / (k0 * k0), 0.0};
  LSOP_HIP(launch_table(op->ktab, op->nx, op->nz, k0 * h, cj1, self, s));
  // spectrum: the row pass writes a transposed px x pz FP64 intermediate
  int st = grow_scratch(op, spectrum_ws_bytes(op));
  if (st) return st;
  LSOP_HIP(launch_spectrum(op->lx, op->lz, op->ktab, op->nx, op->nz, reinterpret_cast<Cx<double>*>(op->scratch),
                           op->gs64, op->gs32, op->tw2x64, op->tw2z64, s));
  op->h = h;
  op->freq = freq_hz;
  op->c0 = c0;
  op->k0 = k0;
  op->ready = true;
  return LSOP_OK;
}

int lsop_set_problem_damped(lsop_op* op, const double* vel_dev, double h, double freq_hz, double c0, double eps,
                            int absorb, void* stream) {
  if (!op) return fail(LSOP_EINVAL, "null operator handle");
  if (op->dims == 3) return fail(LSOP_EUNSUPPORTED, "the dissipative medium is built for 2D operators");
  if (!(eps > 0) || !std::isfinite(eps)) return fail(LSOP_EINVAL, "eps must be positive and finite");
  if (absorb < 0 || 2 * absorb > std::min(op->nx, op->nz)) return fail(LSOP_EINVAL, "absorb outside [0, min(nx, nz) / 2]");
  // the undissipated set-up validates the medium and fills the contrast; the kernel table and spectrum are then
  // replaced by those of the dissipative background
  int st = lsop_set_problem(op, vel_dev, h, freq_hz, c0, stream);
  if (st) return st;
  op->ready = false;
  hipStream_t s = S(stream);
  const size_t n = op->n();
  if (!op->v64) {
    const size_t esz = op->has64() ? sizeof(Cx<double>) : sizeof(Cx<float>);
    void *a = nullptr, *b = nullptr, *c = nullptr;
    if (lib_malloc(&a, sizeof(Cx<double>) * n) != hipSuccess || lib_malloc(&b, sizeof(Cx<float>) * n) != hipSuccess ||
        lib_malloc(&c, esz * (size_t)op->max_vec * n) != hipSuccess) {
      (void)hipGetLastError();
      for (void* p : {a, b, c})
        if (p) (void)hipFree(p);
      return fail(LSOP_ENOMEM, "dissipative operator buffers");
    }
    op->v64 = reinterpret_cast<Cx<double>*>(a);
    op->v32 = reinterpret_cast<Cx<float>*>(b);
    op->vtmp = c;
    op->owned.push_back(a);
    op->owned.push_back(b);
    op->owned.push_back(c);
  }
  LSOP_HIP(launch_damped_potential(op->chi64, op->nx, op->nz, eps, absorb, op->v64, op->v32, s));
  // k^2 = k0^2 + i eps, Re k > 0, Im k > 0; the same disk-integrated kernel with k in place of k0
  using lsop_bessel::C;
  const double pi = lsop_bessel::kPi;
  const double k0 = op->k0;
  const C k = lsop_bessel::c_sqrt(C{k0 * k0, eps});
  const double a = h / std::sqrt(pi);
  const C ka = a * k;
  if (lsop_bessel::c_abs(ka) > 2.0) return fail(LSOP_EINVAL, "grid too coarse for the dissipative kernel: |k a| > 2");
  C j1, y1;
  lsop_bessel::bessel1_small_c(ka, &j1, &y1);
  const C cc = lsop_bessel::c_div(C{0.0, pi * a}, 2.0 * k);
  const C cj1 = cc * j1;
  const C self = cc * C{j1.re - y1.im, j1.im + y1.re} - lsop_bessel::c_div(C{1.0, 0.0}, k * k);
  LSOP_HIP(launch_table_c(op->ktab, op->nx, op->nz, h * k, cj1, self, s));
  if ((st = grow_scratch(op, spectrum_ws_bytes(op)))) return st;
  LSOP_HIP(launch_spectrum(op->lx, op->lz, op->ktab, op->nx, op->nz, reinterpret_cast<Cx<double>*>(op->scratch),
                           op->gs64, op->gs32, op->tw2x64, op->tw2z64, s));
  op->eps = eps;
  op->damped = true;
  op->ready = true;
  return LSOP_OK;
}

int lsop_create3d(int nx, int ny, int nz, int dtype, int max_vec, lsop_op** out) {
  return op_create(nx, nz, dtype, max_vec, nullptr, 0, out, ny);
}

int lsop_set_problem3d(lsop_op* op, const double* vel_dev, double h, double freq_hz, double c0, void* stream) {
  if (!op) return fail(LSOP_EINVAL, "null operator handle");
  if (op->dims != 3) return fail(LSOP_EINVAL, "2D operator: use lsop_set_problem");
  if (!vel_dev) return fail(LSOP_EINVAL, "null velocity");
  if (!(h > 0) || !(freq_hz > 0) || !(c0 > 0) || !std::isfinite(h) || !std::isfinite(freq_hz) || !std::isfinite(c0))
    return fail(LSOP_EINVAL, "h, freq_hz and c0 must be positive and finite");
  const double pi = lsop_bessel::kPi;
  const double w = 2.0 * pi * freq_hz, k0 = w / c0;
  const double a = h * std::cbrt(3.0 / (4.0 * pi));   // radius of the ball of the cell's volume
  const double ka = k0 * a;
  if (ka > 2.0) return fail(LSOP_EINVAL, "grid too coarse: k0 a > 2");
  hipStream_t s = S(stream);
  const size_t n = op->n();
  op->ready = false;
  LSOP_HIP(hipMemsetAsync(op->flag, 0, sizeof(unsigned), s));
  LSOP_HIP(launch_contrast(vel_dev, op->chi64, op->chi32, (int)n, w * w, 1.0 / (c0 * c0), op->flag, s));
  unsigned bad = 0;
  LSOP_HIP(hipMemcpyAsync(&bad, op->flag, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  LSOP_HIP(hipStreamSynchronize(s));
  if (bad) return fail(LSOP_EINVAL, "velocity must be finite and positive");
  // ball-integrated e^{ikr} / (4 pi r): c1 e^{ik0 r} / r off the diagonal, ((1 - i ka) e^{ika} - 1) / k0^2 on it
  double sn, cs;
  sincos(ka, &sn, &cs);
  const double c1 = (sn - ka * cs) / (k0 * k0 * k0);
  const Cx<double> self{(cs + ka * sn - 1.0) / (k0 * k0), (sn - ka * cs) / (k0 * k0)};
  LSOP_HIP(launch_table3(op->ktab, op->nx, op->ny, op->nz, k0, h, c1, self, s));
  int st = grow_scratch(op, spectrum_ws_bytes(op));
  if (st) return st;
  LSOP_HIP(launch_spectrum3(op->lx, op->ly, op->lz, op->ktab, op->nx, op->ny, op->nz,
                            reinterpret_cast<Cx<double>*>(op->tmp), reinterpret_cast<Cx<double>*>(op->scratch),
                            op->gs64, op->gs32, op->tw2x64, op->tw2y64, op->tw2z64, s));
  op->h = h;
  op->freq = freq_hz;
  op->c0 = c0;
  op->k0 = k0;
  op->ready = true;
  return LSOP_OK;
}

int lsop_incident3d(lsop_op* op, const int* src_ijl_host, const double* amp_reim_host, int nsrc, void* psi0_dev,
                    void* stream) {
  int st = check_op(op);
  if (st) return st;
  if (op->dims != 3) return fail(LSOP_EINVAL, "2D operator: use lsop_incident");
  if (nsrc < 0 || (nsrc > 0 && (!src_ijl_host || !psi0_dev))) return fail(LSOP_EINVAL, "bad sources");
  if (nsrc > op->src_cap) return fail(LSOP_EINVAL, "too many sources in one call (max 4096)");
  for (int k = 0; k < nsrc; ++k)
    if (src_ijl_host[3 * k] < 0 || src_ijl_host[3 * k] >= op->nx || src_ijl_host[3 * k + 1] < 0 ||
        src_ijl_host[3 * k + 1] >= op->ny || src_ijl_host[3 * k + 2] < 0 || src_ijl_host[3 * k + 2] >= op->nz)
      return fail(LSOP_EINVAL, "source outside the grid");
  if (nsrc == 0) return LSOP_OK;
  hipStream_t s = S(stream);
  std::vector<Cx<double>> amp(nsrc);
  for (int k = 0; k < nsrc; ++k)
    amp[k] = amp_reim_host ? Cx<double>{amp_reim_host[2 * k], amp_reim_host[2 * k + 1]} : Cx<double>{1.0, 0.0};
  LSOP_HIP(hipStreamSynchronize(s));
  LSOP_HIP(hipMemcpy(op->dsrc, src_ijl_host, sizeof(int) * 3 * (size_t)nsrc, hipMemcpyHostToDevice));
  LSOP_HIP(hipMemcpy(op->damp, amp.data(), sizeof(Cx<double>) * nsrc, hipMemcpyHostToDevice));
  const double inv_dv = 1.0 / (op->h * op->h * op->h);
  if (op->dtype == LSOP_C64)
    LSOP_HIP(launch_incident3<float>(op->ktab, op->dsrc, op->damp, (Cx<float>*)psi0_dev, op->nx, op->ny, op->nz,
                                     nsrc, inv_dv, s));
  else
    LSOP_HIP(launch_incident3<double>(op->ktab, op->dsrc, op->damp, (Cx<double>*)psi0_dev, op->nx, op->ny, op->nz,
                                      nsrc, inv_dv, s));
  return LSOP_OK;
}

int lsop_apply(lsop_op* op, int mode, const void* x_dev, void* y_dev, int nvec, void* stream) {
  int st = check_op(op);
  if (st) return st;
  if (mode < 0 || mode > 3) return fail(LSOP_EINVAL, "bad mode");
  if (nvec < 0 || (nvec > 0 && (!x_dev || !y_dev))) return fail(LSOP_EINVAL, "bad vectors");
  if (op->dtype == LSOP_C64)
    return apply_impl<float>(op, mode, (const Cx<float>*)x_dev, (Cx<float>*)y_dev, nullptr, nullptr, nullptr, nvec,
                             S(stream));
  return apply_impl<double>(op, mode, (const Cx<double>*)x_dev, (Cx<double>*)y_dev, nullptr, nullptr, nullptr, nvec,
                            S(stream));
}

int lsop_residual(lsop_op* op, const void* psi_dev, const void* rhs_dev, void* r_dev, double* rnorm2_dev, int nvec,
                  void* stream) {
  int st = check_op(op);
  if (st) return st;
  if (nvec < 0 || (nvec > 0 && (!psi_dev || !rhs_dev || !r_dev))) return fail(LSOP_EINVAL, "bad vectors");
  hipStream_t s = S(stream);
  if (rnorm2_dev && nvec > 0) LSOP_HIP(hipMemsetAsync(rnorm2_dev, 0, sizeof(double) * nvec, s));
  if (op->dtype == LSOP_C64)
    return apply_impl<float>(op, LSOP_MODE_A, (const Cx<float>*)psi_dev, (Cx<float>*)r_dev,
                             (const Cx<float>*)rhs_dev, rnorm2_dev, nullptr, nvec, s);
  return apply_impl<double>(op, LSOP_MODE_A, (const Cx<double>*)psi_dev, (Cx<double>*)r_dev,
                            (const Cx<double>*)rhs_dev, rnorm2_dev, nullptr, nvec, s);
}

int lsop_incident(lsop_op* op, const int* src_i_host, const int* src_j_host, const double* amp_reim_host, int nsrc,
                  void* psi0_dev, void* stream) {
  int st = check_op(op);
  if (st) return st;
  if (op->dims == 3) return fail(LSOP_EINVAL, "3D operator: use lsop_incident3d");
  if (nsrc < 0 || (nsrc > 0 && (!src_i_host || !src_j_host || !psi0_dev))) return fail(LSOP_EINVAL, "bad sources");
  if (nsrc > op->src_cap) return fail(LSOP_EINVAL, "too many sources in one call (max 4096)");
  for (int k = 0; k < nsrc; ++k)
    if (src_i_host[k] < 0 || src_i_host[k] >= op->nx || src_j_host[k] < 0 || src_j_host[k] >= op->nz)
      return fail(LSOP_EINVAL, "source outside the grid");
  if (nsrc == 0) return LSOP_OK;
  hipStream_t s = S(stream);
  std::vector<int> ij(2 * (size_t)nsrc);
  std::vector<Cx<double>> amp(nsrc);
  for (int k = 0; k < nsrc; ++k) {
    ij[k] = src_i_host[k];
    ij[nsrc + k] = src_j_host[k];
    amp[k] = amp_reim_host ? Cx<double>{amp_reim_host[2 * k], amp_reim_host[2 * k + 1]} : Cx<double>{1.0, 0.0};
  }
  // synchronous copies: the staging buffers are reused by later calls
  LSOP_HIP(hipStreamSynchronize(s));
  LSOP_HIP(hipMemcpy(op->dsrc, ij.data(), sizeof(int) * ij.size(), hipMemcpyHostToDevice));
  LSOP_HIP(hipMemcpy(op->damp, amp.data(), sizeof(Cx<double>) * nsrc, hipMemcpyHostToDevice));
  const double inv_dv = 1.0 / (op->h * op->h);
  if (op->dtype == LSOP_C64)
    LSOP_HIP(launch_incident<float>(op->ktab, op->dsrc, op->dsrc + nsrc, op->damp, (Cx<float>*)psi0_dev, op->nx,
                                    op->nz, nsrc, inv_dv, s));
  else
    LSOP_HIP(launch_incident<double>(op->ktab, op->dsrc, op->dsrc + nsrc, op->damp, (Cx<double>*)psi0_dev, op->nx,
                                     op->nz, nsrc, inv_dv, s));
  return LSOP_OK;
}

int lsop_autotune(lsop_op* op, int nvec, void* stream) {
  int st = check_op(op);
  if (st) return st;
  if (nvec < 1) return fail(LSOP_EINVAL, "nvec must be >= 1");
  const int m = std::min(nvec, op->max_vec);
  if (op->dtype == LSOP_C64) return autotune_cols<float>(op, m, S(stream));
  if ((st = autotune_cols<double>(op, m, S(stream)))) return st;
  return LSOP_OK;
}

int lsop_kernel_table(const lsop_op* op, void* table_dev, void* stream) {
  int st = check_op(op);
  if (st) return st;
  if (!table_dev) return fail(LSOP_EINVAL, "null table");
  LSOP_HIP(hipMemcpyAsync(table_dev, op->ktab, sizeof(Cx<double>) * op->n(), hipMemcpyDeviceToDevice, S(stream)));
  return LSOP_OK;
}

int lsop_info(const lsop_op* op, lsop_op_info* info) {
  if (!op || !info) return fail(LSOP_EINVAL, "null argument");
  info->nx = op->nx;
  info->nz = op->nz;
  info->lx = op->lx;
  info->lz = op->lz;
  info->dtype = op->dtype;
  info->max_vec = op->max_vec;
  info->state_bytes = op->bytes + (op->ws_external ? 0 : op->scratch_bytes);
  info->col_tile = op->col_tile;
  info->ny = op->ny;
  info->ly = op->ly;
  return LSOP_OK;
}

void lsop_destroy(lsop_op* op) {
  if (!op) return;
  (void)hipDeviceSynchronize();
  free_all(op->owned);
  if (op->scratch && !op->ws_external) (void)hipFree(op->scratch);
  delete op;
}

int lsop_workspace_bytes(const lsop_op* op, int nvec, int init, size_t* bytes) {
  if (!op || !bytes) return fail(LSOP_EINVAL, "null argument");
  if (nvec < 0 || init < 0 || init > 3) return fail(LSOP_EINVAL, "bad nvec or init");
  *bytes = std::max(spectrum_ws_bytes(op), series_ws_bytes(op, nvec, init));
  return LSOP_OK;
}

int lsop_attach_workspace(lsop_op* op, void* ws_dev, size_t ws_bytes) {
  if (!op) return fail(LSOP_EINVAL, "null operator handle");
  if (ws_dev && (reinterpret_cast<uintptr_t>(ws_dev) & 255) != 0)
    return fail(LSOP_EINVAL, "workspace must be 256-byte aligned");
  if (op->scratch && !op->ws_external) {
    LSOP_HIP(hipDeviceSynchronize());
    (void)hipFree(op->scratch);
  }
  op->scratch = ws_dev;
  op->scratch_bytes = ws_dev ? ws_bytes : 0;
  op->ws_external = ws_dev != nullptr;
  return LSOP_OK;
}

int lsop_alloc_count(size_t* calls) {
  if (!calls) return fail(LSOP_EINVAL, "null output");
  *calls = g_allocs.load();
  return LSOP_OK;
}

// ------------------------------------------------------------ preconditioner
}  // extern "C"

namespace lsop {
namespace {

// Validates precond_create's parameters and fills the plan fields (no device memory).
int pc_plan(lsop_op* op, const lsop_precond_params* p, lsop_precond* pc) {
  if (!op || !p) return fail(LSOP_EINVAL, "null argument");
  if (p->kind != LSOP_PC_IDENTITY && p->kind != LSOP_PC_LOWRANK && p->kind != LSOP_PC_HODLR &&
      p->kind != LSOP_PC_SCALAR && p->kind != LSOP_PC_GAMMA)
    return fail(LSOP_EINVAL, "bad preconditioner kind");
  if (p->kind == LSOP_PC_SCALAR && (!std::isfinite(p->alpha) || p->alpha == 0.0))
    return fail(LSOP_EINVAL, "alpha must be finite and non-zero");
  if ((p->kind == LSOP_PC_LOWRANK || p->kind == LSOP_PC_HODLR) &&
      (p->rank < 1 || p->rank > 256 || p->power_iters < 0))
    return fail(LSOP_EINVAL, "rank must be in [1, 256] and power_iters >= 0");
  if (p->kind == LSOP_PC_LOWRANK && (p->oversample < 0 || p->rank + p->oversample > 256))
    return fail(LSOP_EINVAL, "oversample must be >= 0 with rank + oversample <= 256");
  if (p->kind != LSOP_PC_LOWRANK && p->oversample != 0)
    return fail(LSOP_EINVAL, "oversampling applies to the low-rank preconditioner only");
  if (p->q_from_level < 0) return fail(LSOP_EINVAL, "q_from_level must be >= 0");
  if (p->min_width < 0) return fail(LSOP_EINVAL, "min_width must be >= 0");
  // Section 2.4's minimum-size rule: no level whose nodes would be narrower than min_width columns
  int levels = p->levels;
  if (p->kind == LSOP_PC_HODLR && p->min_width > 1)
    while (levels > 1 && (op->nx >> levels) < p->min_width) --levels;
  if (p->kind == LSOP_PC_HODLR) {
    if (op->dims == 3) return fail(LSOP_EUNSUPPORTED, "the HODLR tree is built on 2D column strips");
    if (levels < 1 || levels > 16 || op->nx % (1 << levels) != 0)
      return fail(LSOP_EINVAL, "HODLR levels must be >= 1 with nx divisible by 2^levels");
    const size_t nl = (size_t)(op->nx >> levels) * op->nz;
    if (nl % 64 != 0 || nl > 8192)
      return fail(LSOP_EINVAL, "HODLR leaf size (nx / 2^levels) * nz must be a multiple of 64 and at most 8192");
    for (int lv = 0; lv < levels; ++lv)
      if (fft_length_sub(op->nx >> lv) < 0) return fail(LSOP_EUNSUPPORTED, "unsupported HODLR level width");
  }
  pc->op = op;
  pc->kind = p->kind;
  pc->seed = p->seed;
  pc->alpha = p->alpha;
  pc->dt = op->dtype == LSOP_C128 ? LSOP_C128 : LSOP_C64;
  if (p->kind == LSOP_PC_IDENTITY || p->kind == LSOP_PC_SCALAR || p->kind == LSOP_PC_GAMMA) return LSOP_OK;
  pc->rank = p->rank;
  pc->probes = p->kind == LSOP_PC_LOWRANK ? p->rank + p->oversample : p->rank;
  pc->q = p->power_iters;
  pc->q_from = p->kind == LSOP_PC_HODLR ? p->q_from_level : 0;
  const size_t n = op->n();
  pc->tcap = std::max(op->max_vec, pc->probes);
  size_t ks = n / 4096;
  pc->ksplit = (int)std::max<size_t>(1, std::min<size_t>(ks, 256));
  if (p->kind == LSOP_PC_HODLR) {
    pc->levels = levels;
    pc->leaf_w = op->nx >> levels;
    pc->nleaf = 1 << levels;
    const int nl = pc->leaf_w * op->nz;
    pc->maxseg = pc->nleaf;
    pc->ksub_cap = std::max(512, pc->maxseg);
    // leaf workspace, in the leaves' precision (FP32 for complex-FP32 preconditioners): up to 16 GiB of leaf
    // matrices and recursion temporaries per chunk.  Chunks are inverted one after the other, and every launch of
    // the recursion covers the whole chunk: 1024 one-column leaves of 1024 cells at complex FP32 (13.7 GB) take
    // one chunk, so the 64 x 64 base factorisations run 1024 workgroups per launch (128 with 128-leaf chunks,
    // half the CUs idle).
    const size_t esz_leaf = pc->dt == LSOP_C64 ? sizeof(Cx<float>) : sizeof(Cx<double>);
    size_t tmp1 = 0;
    (void)block_inverse_temps(nl, 1, &tmp1);
    const size_t per_leaf = ((size_t)nl * nl + tmp1) * esz_leaf;
    pc->leaf_chunk = (int)std::max<size_t>(1, std::min<size_t>(pc->nleaf, ((size_t)16 << 30) / per_leaf));
    if (const char* lc = getenv("LSOP_HODLR_LEAF_CHUNK"))  // smaller chunks (exercises the chunked leaf build)
      pc->leaf_chunk = std::max(1, std::min(pc->leaf_chunk, atoi(lc)));
    size_t lw = 0;
    (void)block_inverse_temps(nl, pc->leaf_chunk, &lw);
    lw += (size_t)pc->leaf_chunk * nl * nl;
    // allocated in complex-double units
    pc->lwork_elems = (lw * esz_leaf + sizeof(Cx<double>) - 1) / sizeof(Cx<double>);
    pc->lev.resize(levels);
    // the zero-padded sampling form on every level (both forms give the same samples; compared in tests)
    const char* pad_env = getenv("LSOP_HODLR_PADDED_SAMPLING");
    const bool padded_sampling = pad_env && atoi(pad_env) != 0;
    for (int lv = 0; lv < levels; ++lv) {
      hodlr_level& L = pc->lev[lv];
      L.width = op->nx >> lv;
      // between the two halves of a node only the x-lags 1 .. width - 1 occur, so a circular convolution of
      // period width (x-transform pair of length width / 2) is exact where that length is one the FFT engine has,
      // or 1 (width 2: no transform, one spectrum factor per z-frequency)
      const int h = L.width / 2;
      L.half = L.width % 2 == 0 && h >= 1 && (h == 1 || fft_length_sub(h) == h) && !padded_sampling;
      L.lx = L.half ? h : fft_length_sub(L.width);
    }
  }
  return LSOP_OK;
}

// Every device buffer of a preconditioner's state, in one fixed order (the size query walks the same list).
int pc_buffers(lsop_precond* pc, Alloc& a) {
  if (pc->kind == LSOP_PC_IDENTITY || pc->kind == LSOP_PC_SCALAR || pc->kind == LSOP_PC_GAMMA) return LSOP_OK;
  const lsop_op* op = pc->op;
  const size_t n = op->n();
  const size_t esz = pc->dt == LSOP_C128 ? sizeof(Cx<double>) : sizeof(Cx<float>);
  const int r = pc->rank, l = pc->probes;
  int st = 0;
  if (pc->kind == LSOP_PC_LOWRANK) {
    st |= dev_alloc(a, &pc->U, esz * l * n);
    st |= dev_alloc(a, &pc->W, esz * l * n);
    st |= dev_alloc(a, &pc->Y, esz * l * n);
    st |= dev_alloc(a, &pc->Z, sizeof(Cx<double>) * r * r);
    // small: G / M (l*l), X / LU work (2 l*l), T1, T2 (l * tcap each)
    st |= dev_alloc(a, &pc->small, sizeof(Cx<double>) * ((size_t)3 * l * l + (size_t)2 * l * pc->tcap));
    pc->part_cap = (size_t)pc->ksplit * l * pc->tcap;
    st |= dev_alloc(a, &pc->part, sizeof(Cx<double>) * pc->part_cap);
    st |= dev_alloc(a, &pc->dflag, 256);
    if (l > r) {
      st |= dev_alloc(a, &pc->Q2, esz * l * n);
      st |= dev_alloc(a, &pc->svdw, sizeof(Cx<double>) * ((size_t)3 * l * l + (size_t)2 * l * r));
    }
    return st ? LSOP_ENOMEM : LSOP_OK;
  }
  // HODLR: the leaf workspace and the sampling buffers U, Y live only during precond_build
  const int nl = pc->leaf_w * op->nz;
  st |= dev_alloc(a, &pc->dinv, esz * (size_t)pc->nleaf * nl * nl);
  st |= dev_alloc(a, &pc->hy, esz * (size_t)pc->tcap * n);
  const size_t small = (size_t)pc->maxseg * r * pc->tcap;
  st |= dev_alloc(a, &pc->hG, sizeof(Cx<double>) * small);
  st |= dev_alloc(a, &pc->hX, sizeof(Cx<double>) * small);
  if (pc->dt == LSOP_C64) {
    st |= dev_alloc(a, &pc->hG32, sizeof(Cx<float>) * small);
    st |= dev_alloc(a, &pc->hX32, sizeof(Cx<float>) * small);
  }
  // node cores: recursion temporaries (< r^2 per node), S S^{-1} (r^2 per node), pivoted fallback work (2 r^2)
  st |= dev_alloc(a, &pc->hK, sizeof(Cx<double>) * ((size_t)(pc->maxseg / 2) * 3 * r * r + 2 * (size_t)r * r));
  pc->part_cap = (size_t)pc->ksub_cap * r * pc->tcap;
  st |= dev_alloc(a, &pc->part, sizeof(Cx<double>) * pc->part_cap);
  st |= dev_alloc(a, &pc->hflag, sizeof(int) * (4 * (size_t)pc->maxseg + pc->leaf_chunk + 64));
  for (int lv = 0; lv < pc->levels; ++lv) {
    hodlr_level& L = pc->lev[lv];
    const int nodes = 1 << lv;
    st |= dev_alloc(a, &L.V, esz * r * n);
    st |= dev_alloc(a, &L.Wp, esz * r * n);
    st |= dev_alloc(a, &L.kinv, sizeof(Cx<double>) * (size_t)nodes * 4 * r * r);
    if (pc->dt == LSOP_C64) st |= dev_alloc(a, &L.kinv32, sizeof(Cx<float>) * (size_t)nodes * 4 * r * r);
    const size_t gsz = (size_t)2 * op->pz() * L.lx;
    if (pc->dt == LSOP_C128) st |= dev_alloc(a, &L.gs64, sizeof(Cx<double>) * gsz);
    else st |= dev_alloc(a, &L.gs32, sizeof(Cx<float>) * gsz);
    st |= dev_alloc(a, &L.tw64, sizeof(Cx<double>) * 2 * L.lx);
    st |= dev_alloc(a, &L.tw32, sizeof(Cx<float>) * 2 * L.lx);
  }
  return st ? LSOP_ENOMEM : LSOP_OK;
}

// Transient workspace of precond_build: HODLR sampling buffers and leaf workspace (or the sub-domain
// spectrum intermediate, if larger); none for the other kinds.
size_t pc_build_ws_bytes(const lsop_precond* pc) {
  if (pc->kind != LSOP_PC_HODLR) return 0;
  const size_t n = pc->op->n();
  const size_t esz = pc->dt == LSOP_C128 ? sizeof(Cx<double>) : sizeof(Cx<float>);
  size_t spec = 0;
  for (const hodlr_level& L : pc->lev) spec = std::max(spec, sizeof(Cx<double>) * (size_t)(2 * L.lx) * pc->op->pz());
  return std::max(spec, 2 * align_up(esz * pc->rank * n) + align_up(sizeof(Cx<double>) * pc->lwork_elems));
}

int pc_create(lsop_op* op, const lsop_precond_params* p, void* state, size_t state_bytes, lsop_precond** out) {
  if (!out) return fail(LSOP_EINVAL, "null output handle");
  *out = nullptr;
  lsop_precond* pc = new lsop_precond();
  int st = pc_plan(op, p, pc);
  if (st) {
    delete pc;
    return st;
  }
  if (pc->kind == LSOP_PC_IDENTITY || pc->kind == LSOP_PC_SCALAR || pc->kind == LSOP_PC_GAMMA) pc->built = true;
  Alloc a;
  a.owned = &pc->owned;
  a.bytes = &pc->bytes;
  if (state) {
    a.base = reinterpret_cast<char*>(state);
    a.cap = state_bytes;
    pc->state_external = true;
  }
  st = pc_buffers(pc, a);
  for (int lv = 0; lv < pc->levels && !st; ++lv) {
    hodlr_level& L = pc->lev[lv];
    std::vector<Cx<double>> w = twiddles(L.lx);
    std::vector<Cx<float>> w32(w.size());
    for (size_t t = 0; t < w.size(); ++t) w32[t] = ccast<float>(w[t]);
    if (hipMemcpy(L.tw64, w.data(), sizeof(Cx<double>) * w.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L.tw32, w32.data(), sizeof(Cx<float>) * w32.size(), hipMemcpyHostToDevice) != hipSuccess)
      st = fail(LSOP_EHIP, "twiddle upload failed");
  }
  if (st) {
    free_all(pc->owned);
    delete pc;
    return st;
  }
  *out = pc;
  return LSOP_OK;
}

}  // namespace
}  // namespace lsop

extern "C" {

int precond_create(lsop_op* op, const lsop_precond_params* p, lsop_precond** out) {
  return pc_create(op, p, nullptr, 0, out);
}

int precond_create_in(lsop_op* op, const lsop_precond_params* p, void* state_dev, size_t state_bytes,
                      lsop_precond** out) {
  if (!state_dev || (reinterpret_cast<uintptr_t>(state_dev) & 255) != 0)
    return fail(LSOP_EINVAL, "state buffer must be non-null and 256-byte aligned");
  return pc_create(op, p, state_dev, state_bytes, out);
}

int precond_state_bytes(const lsop_op* op, const lsop_precond_params* p, size_t* state, size_t* build_ws) {
  if (!state || !build_ws) return fail(LSOP_EINVAL, "null output");
  lsop_precond pc;
  int st = pc_plan(const_cast<lsop_op*>(op), p, &pc);
  if (st) return st;
  size_t total = 0;
  Alloc a;
  a.bytes = &total;
  a.count_only = true;
  (void)pc_buffers(&pc, a);
  *state = total;
  *build_ws = pc_build_ws_bytes(&pc);
  return LSOP_OK;
}

int precond_build(lsop_precond* pc, const void* omega_dev, void* stream) {
  if (!pc) return fail(LSOP_EINVAL, "null preconditioner");
  int st = check_op(pc->op);
  if (st) return st;
  if (pc->kind == LSOP_PC_IDENTITY || pc->kind == LSOP_PC_SCALAR) return LSOP_OK;
  if (pc->kind == LSOP_PC_GAMMA)
    return pc->op->damped ? LSOP_OK : fail(LSOP_EINVAL, "H = gamma needs an operator set by lsop_set_problem_damped");
  if (pc->kind == LSOP_PC_HODLR && pc->op->damped)
    return fail(LSOP_EUNSUPPORTED, "the HODLR build samples the undissipated contrast; not for a damped operator");
  pc->built = false;
  if (pc->kind == LSOP_PC_HODLR) {
    if (pc->dt == LSOP_C128) return hodlr_build<double>(pc, (const double*)omega_dev, S(stream));
    return hodlr_build<float>(pc, (const double*)omega_dev, S(stream));
  }
  if (pc->dt == LSOP_C128) return build_impl<double>(pc, (const double*)omega_dev, S(stream));
  return build_impl<float>(pc, (const double*)omega_dev, S(stream));
}

int precond_build_batch(lsop_precond* const* pcs, int count, int streams) {
  if (count < 0 || (count > 0 && !pcs)) return fail(LSOP_EINVAL, "bad preconditioner list");
  if (streams < 1 || streams > 16) return fail(LSOP_EINVAL, "streams must be in 1..16");
  std::vector<int> order;
  for (int i = 0; i < count; ++i) {
    if (!pcs[i]) return fail(LSOP_EINVAL, "null preconditioner in the list");
    for (int j = 0; j < i; ++j)
      if (pcs[j]->op == pcs[i]->op) return fail(LSOP_EINVAL, "two preconditioners of one operator in one batch build");
    order.push_back(i);
  }
  // largest grids first, handed out one at a time to the workers (longest-processing-time order)
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return pcs[a]->op->n() > pcs[b]->op->n(); });
  LSOP_HIP(hipDeviceSynchronize());
  const int nw = std::max(1, std::min(streams, count));
  std::atomic<int> next{0};
  std::vector<int> status(nw, LSOP_OK);
  std::vector<std::string> msg(nw);
  auto worker = [&](int w) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      status[w] = LSOP_EHIP;
      msg[w] = "stream creation failed";
      return;
    }
    for (int k; (k = next.fetch_add(1)) < count;) {
      const int r = precond_build(pcs[order[k]], nullptr, st);
      if (r != LSOP_OK && status[w] == LSOP_OK) {
        status[w] = r;
        msg[w] = lsop_last_error();
      }
    }
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < nw; ++w) pool.emplace_back(worker, w);
  worker(0);
  for (auto& t : pool) t.join();
  for (int w = 0; w < nw; ++w)
    if (status[w] != LSOP_OK) return fail(status[w], msg[w]);
  return LSOP_OK;
}

int precond_apply(lsop_precond* pc, const void* x_dev, void* y_dev, int nvec, void* stream) {
  if (!pc) return fail(LSOP_EINVAL, "null preconditioner");
  if (!pc->built) return fail(LSOP_EINVAL, "preconditioner not built");
  if (nvec < 0 || (nvec > 0 && (!x_dev || !y_dev))) return fail(LSOP_EINVAL, "bad vectors");
  if (pc->dt == LSOP_C128)
    return pc_apply_impl<double>(pc, (const Cx<double>*)x_dev, (Cx<double>*)y_dev, nullptr, nvec, false, S(stream));
  return pc_apply_impl<float>(pc, (const Cx<float>*)x_dev, (Cx<float>*)y_dev, nullptr, nvec, false, S(stream));
}

int precond_depth(const lsop_precond* pc, int* levels) {
  if (!pc || !levels) return fail(LSOP_EINVAL, "null argument");
  *levels = pc->kind == LSOP_PC_HODLR ? pc->levels : 0;
  return LSOP_OK;
}

int precond_info(const lsop_precond* pc, int* rank, double* compression, size_t* bytes) {
  if (!pc) return fail(LSOP_EINVAL, "null preconditioner");
  const int r = pc->kind == LSOP_PC_IDENTITY ? 0 : pc->kept;
  if (rank) *rank = r;
  const double n = (double)pc->op->n();
  if (compression) {
    if (pc->kind == LSOP_PC_HODLR) {
      const double nl = (double)pc->leaf_w * pc->op->nz;
      *compression = (pc->nleaf * nl * nl + 2.0 * pc->levels * pc->rank * n) / (n * n);
    } else {
      *compression = 2.0 * r / n;
    }
  }
  if (bytes) *bytes = pc->bytes;
  return LSOP_OK;
}

void precond_destroy(lsop_precond* pc) {
  if (!pc) return;
  (void)hipDeviceSynchronize();
  free_all(pc->owned);
  delete pc;
}

// ------------------------------------------------------------------ series
// series_solve with its workspace at byte offset `off` of the operator's scratch (the bytes before it hold the
// right-hand sides of series_solve_sources)
static int series_solve_at(lsop_op* op, lsop_precond* pc, const void* rhs_dev, void* psi_dev, int nvec,
                           const lsop_solve_params* p, lsop_solve_info* info, void* stream, size_t off) {
  int st = check_op(op);
  if (st) return st;
  if (!p || !info) return fail(LSOP_EINVAL, "null params or info");
  if (nvec < 1 || !rhs_dev || !psi_dev) return fail(LSOP_EINVAL, "bad vectors");
  if (!(p->tol > 0) || p->max_iter < 0) return fail(LSOP_EINVAL, "tol must be > 0 and max_iter >= 0");
  if (p->init < 0 || p->init > 3) return fail(LSOP_EINVAL, "bad init");
  if (pc && pc->op != op) return fail(LSOP_EINVAL, "preconditioner belongs to another operator");
  if (pc && !pc->built) return fail(LSOP_EINVAL, "preconditioner not built");
  lsop_precond* pcu = (pc && pc->kind != LSOP_PC_IDENTITY) ? pc : nullptr;
  hipStream_t s = S(stream);
  const size_t n = op->n();
  for (int v = 0; v < nvec; ++v) info[v] = lsop_solve_info{0, 0, INFINITY, LSOP_NOT_CONVERGED, INFINITY};
  if (op->dtype != LSOP_MIXED) {
    const size_t esz = op->dtype == LSOP_C64 ? sizeof(Cx<float>) : sizeof(Cx<double>);
    const size_t vb = align_up(esz * n * nvec);
    if ((st = grow_scratch(op, off + series_ws_bytes(op, nvec, p->init)))) return st;
    char* base = (char*)op->scratch + off;
    void* r = base;
    double* dn = (double*)(base + vb);
    int* dv = (int*)((char*)dn + align_up(sizeof(double) * nvec));
    void* alt = p->init == LSOP_INIT_BEST ? (char*)dv + align_up(sizeof(int) * nvec) : nullptr;
    if (op->dtype == LSOP_C64)
      st = series_impl<float>(op, pcu, (const Cx<float>*)rhs_dev, (Cx<float>*)psi_dev, nvec, p->tol, p->max_iter,
                              p->init, {}, info, (Cx<float>*)r, dn, dv, s, (Cx<float>*)alt);
    else
      st = series_impl<double>(op, pcu, (const Cx<double>*)rhs_dev, (Cx<double>*)psi_dev, nvec, p->tol, p->max_iter,
                               p->init, {}, info, (Cx<double>*)r, dn, dv, s, (Cx<double>*)alt);
    if (st) return st;
    return overall_status(info, nvec);
  }
  // ---- mixed precision: iterative refinement (outer FP64, inner FP32 series)
  const int refine_max = p->refine_max > 0 ? p->refine_max : 8;
  const double inner_tol = p->inner_tol > 0 ? p->inner_tol : 1e-5;
  if ((st = grow_scratch(op, off + series_ws_bytes(op, nvec, p->init)))) return st;
  char* w32 = (char*)op->scratch + off + refine_ws_bytes(n, nvec);
  auto inner = [&](const Cx<float>* rhs32, Cx<float>* d32, const std::vector<int>& active, lsop_solve_info* inf,
                   double* dn, int* dv) {
    return series_impl<float>(op, pcu, rhs32, d32, nvec, inner_tol, p->max_iter, LSOP_INIT_H_RHS, active, inf,
                              (Cx<float>*)w32, dn, dv, s);
  };
  return refine_impl(op, (const Cx<double>*)rhs_dev, (Cx<double>*)psi_dev, nvec, p->tol, refine_max, p->init, info,
                     (char*)op->scratch + off, s, inner);
}

int series_solve(lsop_op* op, lsop_precond* pc, const void* rhs_dev, void* psi_dev, int nvec,
                 const lsop_solve_params* p, lsop_solve_info* info, void* stream) {
  return series_solve_at(op, pc, rhs_dev, psi_dev, nvec, p, info, stream, 0);
}

// bytes of the incident fields series_solve_sources keeps in the workspace ahead of the series' own
static size_t sources_rhs_bytes(const lsop_op* op, int nsrc) {
  const size_t esz = op->dtype == LSOP_C64 ? sizeof(Cx<float>) : sizeof(Cx<double>);
  return align_up(esz * op->n() * (size_t)nsrc);
}

int series_sources_workspace_bytes(const lsop_op* op, int nsrc, int init, size_t* bytes) {
  if (!op || !bytes) return fail(LSOP_EINVAL, "null argument");
  if (nsrc < 0 || init < 0 || init > 3) return fail(LSOP_EINVAL, "bad nsrc or init");
  *bytes = sources_rhs_bytes(op, nsrc) + series_ws_bytes(op, nsrc, init);
  return LSOP_OK;
}

int series_solve_sources(lsop_op* op, lsop_precond* pc, const int* src_i_host, const int* src_j_host,
                         const double* amp_reim_host, int nsrc, void* psi_dev, const lsop_solve_params* p,
                         lsop_solve_info* info, void* stream) {
  int st = check_op(op);
  if (st) return st;
  if (op->dims == 3) return fail(LSOP_EINVAL, "3D operator: use lsop_incident3d and series_solve");
  if (!p || !info) return fail(LSOP_EINVAL, "null params or info");
  if (nsrc < 1 || !src_i_host || !src_j_host || !psi_dev) return fail(LSOP_EINVAL, "bad sources");
  if (p->init < 0 || p->init > 3) return fail(LSOP_EINVAL, "bad init");
  const size_t rb = sources_rhs_bytes(op, nsrc);
  // the whole workspace first: a library-owned workspace that grew later would lose the incident fields
  if ((st = grow_scratch(op, rb + series_ws_bytes(op, nsrc, p->init)))) return st;
  if ((st = lsop_incident(op, src_i_host, src_j_host, amp_reim_host, nsrc, op->scratch, stream))) return st;
  return series_solve_at(op, pc, op->scratch, psi_dev, nsrc, p, info, stream, rb);
}

static int gmres_ws_query(const lsop_op* op, int nvec, int restart, size_t* bytes);

int gmres_solve(lsop_op* op, lsop_precond* pc, const void* rhs_dev, void* psi_dev, int nvec,
                const lsop_gmres_params* p, lsop_solve_info* info, void* stream) {
  int st = check_op(op);
  if (st) return st;
  if (!p || !info) return fail(LSOP_EINVAL, "null params or info");
  if (nvec < 1 || !rhs_dev || !psi_dev) return fail(LSOP_EINVAL, "bad vectors");
  if (!(p->tol > 0) || p->max_iter < 0 || p->restart < 1 || p->restart > 200)
    return fail(LSOP_EINVAL, "tol must be > 0, max_iter >= 0 and restart in [1, 200]");
  if (p->init != LSOP_INIT_H_RHS && p->init != LSOP_INIT_ZERO && p->init != LSOP_INIT_USER)
    return fail(LSOP_EINVAL, "GMRES starts from H psi0, zero or the caller's psi");
  if (pc && pc->op != op) return fail(LSOP_EINVAL, "preconditioner belongs to another operator");
  if (pc && !pc->built) return fail(LSOP_EINVAL, "preconditioner not built");
  lsop_precond* pcu = (pc && pc->kind != LSOP_PC_IDENTITY) ? pc : nullptr;
  hipStream_t s = S(stream);
  const size_t n = op->n();
  size_t need = 0;
  if ((st = gmres_ws_query(op, nvec, p->restart, &need))) return st;
  if ((st = grow_scratch(op, need))) return st;
  for (int v = 0; v < nvec; ++v) info[v] = lsop_solve_info{0, 0, INFINITY, LSOP_NOT_CONVERGED, INFINITY};
  if (op->dtype == LSOP_C64) {
    if ((st = gmres_impl<float>(op, pcu, (const Cx<float>*)rhs_dev, (Cx<float>*)psi_dev, nvec, p->tol, p->restart,
                                p->max_iter, p->init, {}, info, (char*)op->scratch, s)))
      return st;
    return overall_status(info, nvec);
  }
  if (op->dtype == LSOP_C128) {
    if ((st = gmres_impl<double>(op, pcu, (const Cx<double>*)rhs_dev, (Cx<double>*)psi_dev, nvec, p->tol,
                                 p->restart, p->max_iter, p->init, {}, info, (char*)op->scratch, s)))
      return st;
    return overall_status(info, nvec);
  }
  // mixed: FP64 refinement around complex-FP32 GMRES (inner tolerance inner_tol, default 1e-5)
  const double inner_tol = p->inner_tol > 0 ? p->inner_tol : 1e-5;
  const int refine_max = p->refine_max > 0 ? p->refine_max : 8;
  char* gws = (char*)op->scratch + refine_ws_bytes(n, nvec);
  auto inner = [&](const Cx<float>* rhs32, Cx<float>* d32, const std::vector<int>& active, lsop_solve_info* inf,
                   double*, int*) {
    return gmres_impl<float>(op, pcu, rhs32, d32, nvec, inner_tol, p->restart, p->max_iter, LSOP_INIT_ZERO, active,
                             inf, gws, s);
  };
  return refine_impl(op, (const Cx<double>*)rhs_dev, (Cx<double>*)psi_dev, nvec, p->tol, refine_max,
                     p->init == LSOP_INIT_USER ? LSOP_INIT_USER : LSOP_INIT_ZERO, info, (char*)op->scratch, s, inner);
}

static int gmres_ws_query(const lsop_op* op, int nvec, int restart, size_t* bytes) {
  const size_t n = op->n();
  if (op->dtype == LSOP_C64) *bytes = gmres_ws_bytes(n, nvec, restart, sizeof(Cx<float>));
  else if (op->dtype == LSOP_C128) *bytes = gmres_ws_bytes(n, nvec, restart, sizeof(Cx<double>));
  else *bytes = refine_ws_bytes(n, nvec) + gmres_ws_bytes(n, nvec, restart, sizeof(Cx<float>));
  return LSOP_OK;
}

int gmres_workspace_bytes(const lsop_op* op, int nvec, int restart, size_t* bytes) {
  if (!op || !bytes) return fail(LSOP_EINVAL, "null argument");
  if (nvec < 0 || restart < 1 || restart > 200) return fail(LSOP_EINVAL, "bad nvec or restart");
  return gmres_ws_query(op, nvec, restart, bytes);
}

// ------------------------------------------------------------------ frequency sweep
// Section 3.1: integer frequencies lowest first; a preconditioner per frequency; at most max_iter iterations of
// the series; on failure the preconditioner is rebuilt with a larger rank and the series restarted from psi0;
// when a frequency needed more than escalate_above iterations, the next one starts at a larger rank.
static Cx<double> ricker_amp(double f, double fc) {
  // Fourier transform of the Ricker wavelet (1 - 2 pi^2 fc^2 t'^2) exp(-pi^2 fc^2 t'^2), t' = t - 1/fc:
  // (2 / sqrt(pi)) f^2 / fc^3 exp(-f^2 / fc^2) times the delay phase exp(-i 2 pi f / fc)
  const double pi = lsop_bessel::kPi;
  const double a = 2.0 / std::sqrt(pi) * f * f / (fc * fc * fc) * std::exp(-f * f / (fc * fc));
  const double ph = -2.0 * pi * f / fc;
  return Cx<double>{a * std::cos(ph), a * std::sin(ph)};
}

int lsop_sweep(lsop_op* op, const double* vel_dev, double h, double c0, const double* freqs, int nfreq,
               const lsop_precond_params* pc0, const lsop_sweep_params* sp, const int* src_i, const int* src_j,
               int nsrc, void* psi_dev, lsop_sweep_info* info, void* stream) {
  if (!op || !vel_dev || !freqs || !pc0 || !sp || !src_i || !src_j || !psi_dev || !info)
    return fail(LSOP_EINVAL, "null argument");
  if (nfreq < 1 || nsrc < 1) return fail(LSOP_EINVAL, "nfreq and nsrc must be >= 1");
  for (int k = 0; k < nfreq; ++k)
    if (!(freqs[k] > 0) || (k > 0 && !(freqs[k] > freqs[k - 1])))
      return fail(LSOP_EINVAL, "frequencies must be positive and increasing (lowest first)");
  if (pc0->kind != LSOP_PC_LOWRANK && pc0->kind != LSOP_PC_HODLR)
    return fail(LSOP_EINVAL, "the sweep escalates the rank of a low-rank or HODLR preconditioner");
  if (!(sp->tol > 0) || sp->max_iter < 1 || sp->rank_step < 1 || sp->max_rebuilds < 0 || sp->escalate_above < 0 ||
      sp->ricker_fc < 0 || !std::isfinite(sp->ricker_fc))
    return fail(LSOP_EINVAL, "bad sweep parameters");
  const int rank_cap = std::min(256 - (pc0->kind == LSOP_PC_LOWRANK ? pc0->oversample : 0),
                                sp->rank_max > 0 ? sp->rank_max : 256);
  if (pc0->rank < 1 || pc0->rank > rank_cap) return fail(LSOP_EINVAL, "initial rank outside [1, rank_max]");
  for (int k = 0; k < nsrc; ++k)
    if (src_i[k] < 0 || src_i[k] >= op->nx || src_j[k] < 0 || src_j[k] >= op->nz)
      return fail(LSOP_EINVAL, "source outside the grid");
  const size_t esz = op->dtype == LSOP_C64 ? sizeof(Cx<float>) : sizeof(Cx<double>);
  const size_t vstride = esz * op->n() * nsrc;
  lsop_precond_params pp = *pc0;
  std::vector<double> amp(2 * (size_t)nsrc);
  std::vector<lsop_solve_info> si(nsrc);
  lsop_solve_params prm{sp->tol, sp->max_iter, LSOP_INIT_H_RHS, 0, 0.0};
  int overall = LSOP_OK;
  // the incident fields of the current frequency live in the caller's output slice of the *next* frequency
  // until that one is solved; the last frequency uses a small library buffer
  void* last_rhs = nullptr;
  int st = 0;
  for (int k = 0; k < nfreq; ++k) {
    info[k] = lsop_sweep_info{freqs[k], pp.rank, 0, 0, LSOP_NOT_CONVERGED, INFINITY};
    if ((st = lsop_set_problem(op, vel_dev, h, freqs[k], c0, stream))) return st;
    const Cx<double> a = sp->ricker_fc > 0 ? ricker_amp(freqs[k], sp->ricker_fc) : Cx<double>{1.0, 0.0};
    for (int q = 0; q < nsrc; ++q) {
      amp[2 * q] = a.re;
      amp[2 * q + 1] = a.im;
    }
    char* psi_k = (char*)psi_dev + (size_t)k * vstride;
    void* rhs = nullptr;
    if (k + 1 < nfreq) {
      rhs = (char*)psi_dev + (size_t)(k + 1) * vstride;
    } else {
      if (!last_rhs && lib_malloc(&last_rhs, vstride) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LSOP_ENOMEM, "sweep: incident-field buffer");
      }
      rhs = last_rhs;
    }
    if ((st = lsop_incident(op, src_i, src_j, amp.data(), nsrc, rhs, stream))) break;
    for (int rebuild = 0;; ++rebuild) {
      for (lsop_solve_info& x : si) x = lsop_solve_info{0, 0, INFINITY, LSOP_NOT_CONVERGED, INFINITY};
      lsop_precond* pc = nullptr;
      if ((st = precond_create(op, &pp, &pc))) break;
      st = precond_build(pc, nullptr, stream);
      int ss = st;
      if (!st) ss = series_solve(op, pc, rhs, psi_k, nsrc, &prm, si.data(), stream);
      precond_destroy(pc);
      if (st && st != LSOP_ESINGULAR) break;  // a singular core counts as a failed build: raise the rank
      st = 0;
      int itmax = 0;
      double resmax = 0.0;
      for (const lsop_solve_info& x : si) {
        itmax = std::max(itmax, x.iters);
        resmax = std::max(resmax, x.rel_residual);
      }
      info[k].rank = pp.rank;
      info[k].rebuilds = rebuild;
      info[k].iters_max = itmax;
      info[k].rel_residual_max = resmax;
      info[k].status = ss;
      if (ss == LSOP_OK) {
        if (itmax > sp->escalate_above) pp.rank = std::min(rank_cap, pp.rank + sp->rank_step);
        break;
      }
      if (rebuild >= sp->max_rebuilds || pp.rank >= rank_cap) break;
      pp.rank = std::min(rank_cap, pp.rank + sp->rank_step);  // rebuild with a larger rank, restart from psi0
    }
    if (st) break;
    if (info[k].status != LSOP_OK && overall == LSOP_OK) overall = info[k].status;
  }
  if (last_rhs) {
    (void)hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    (void)hipFree(last_rhs);
  }
  return st ? st : overall;
}

// ------------------------------------------------------------------ batches
int lsop_batch_create(int count, lsop_op* const* ops, lsop_batch** out) {
  if (!out) return fail(LSOP_EINVAL, "null output handle");
  *out = nullptr;
  if (count < 1 || !ops) return fail(LSOP_EINVAL, "count must be >= 1 with an operator array");
  int dt = -1;
  for (int i = 0; i < count; ++i) {
    int st = check_op(ops[i]);
    if (st) return st;
    if (ops[i]->dtype == LSOP_MIXED) return fail(LSOP_EUNSUPPORTED, "batches take complex float or double operators");
    if (ops[i]->damped) return fail(LSOP_EUNSUPPORTED, "batches take undissipated operators");
    if (ops[i]->dims == 3) return fail(LSOP_EUNSUPPORTED, "batches take 2D operators");
    if (dt >= 0 && ops[i]->dtype != dt) return fail(LSOP_EINVAL, "all operators of a batch must share one dtype");
    dt = ops[i]->dtype;
  }
  lsop_batch* b = new lsop_batch();
  b->count = count;
  b->dtype = dt;
  b->ops.assign(ops, ops + count);
  b->group_of.assign(count, -1);
  for (int i = 0; i < count; ++i) {
    const lsop_op* op = ops[i];
    int g = -1;
    for (size_t k = 0; k < b->groups.size(); ++k) {
      const auto& G = b->groups[k];
      if (G.nx == op->nx && G.nz == op->nz && G.lx == op->lx && G.lz == op->lz) g = (int)k;
    }
    if (g < 0) {
      lsop_batch::Group G;
      G.nx = op->nx;
      G.nz = op->nz;
      G.lx = op->lx;
      G.lz = op->lz;
      G.col_tile = op->col_tile;
      b->groups.push_back(G);
      g = (int)b->groups.size() - 1;
    }
    b->groups[g].members.push_back(i);
    b->group_of[i] = g;
  }
  *out = b;
  return LSOP_OK;
}

static int check_batch_vectors(const lsop_batch* b, const void* const* x, void* const* y, const int* nvec) {
  for (const lsop_op* op : b->ops)
    if (op->damped) return fail(LSOP_EUNSUPPORTED, "a batch member was set up as a dissipative operator");
  if (!b) return fail(LSOP_EINVAL, "null batch");
  if (!nvec || !x || !y) return fail(LSOP_EINVAL, "null vector arrays");
  for (int i = 0; i < b->count; ++i) {
    if (nvec[i] < 0) return fail(LSOP_EINVAL, "nvec must be >= 0");
    if (nvec[i] > 0 && (!x[i] || !y[i])) return fail(LSOP_EINVAL, "null vectors for an instance");
    if (!b->ops[i]->ready) return fail(LSOP_EINVAL, "an operator of the batch has no problem set");
  }
  return LSOP_OK;
}

int lsop_batch_apply(lsop_batch* b, int mode, const void* const* x_dev, void* const* y_dev, const int* nvec,
                     void* stream) {
  int st = check_batch_vectors(b, x_dev, y_dev, nvec);
  if (st) return st;
  if (mode < 0 || mode > 3) return fail(LSOP_EINVAL, "bad mode");
  if (b->dtype == LSOP_C64)
    return batch_apply_impl<float>(b, mode, reinterpret_cast<const Cx<float>* const*>(x_dev),
                                   reinterpret_cast<Cx<float>* const*>(y_dev), nvec, S(stream));
  return batch_apply_impl<double>(b, mode, reinterpret_cast<const Cx<double>* const*>(x_dev),
                                  reinterpret_cast<Cx<double>* const*>(y_dev), nvec, S(stream));
}

int lsop_batch_autotune(lsop_batch* b, void* stream) {
  if (!b) return fail(LSOP_EINVAL, "null batch");
  // one tuning per shape group (the tile depends on the column length and the slot count), cached by shape
  static std::vector<std::array<int, 5>> cache;  // dtype, lx, lz, slots bucket, tile
  for (auto& G : b->groups) {
    lsop_op* op0 = b->ops[G.members[0]];
    const int m = std::min(op0->max_vec, 64);
    const int bucket = 31 - __builtin_clz((unsigned)std::max(1, m));
    int tile = -1;
    for (const auto& c : cache)
      if (c[0] == b->dtype && c[1] == G.lx && c[2] == G.lz && c[3] == bucket) tile = c[4];
    if (tile < 0) {
      int st = lsop_autotune(op0, m, stream);
      if (st) return st;
      tile = op0->col_tile;
      cache.push_back({b->dtype, G.lx, G.lz, bucket, tile});
    }
    G.col_tile = tile;
  }
  return LSOP_OK;
}

int lsop_batch_solve(lsop_batch* b, lsop_precond* const* pcs, const void* const* rhs_dev, void* const* psi_dev,
                     const int* nvec, const lsop_solve_params* p, int use_graph, lsop_solve_info* info, void* stream) {
  int st = check_batch_vectors(b, rhs_dev, psi_dev, nvec);
  if (st) return st;
  if (!p || !info) return fail(LSOP_EINVAL, "null params or info");
  if (!(p->tol > 0) || p->max_iter < 0) return fail(LSOP_EINVAL, "tol must be > 0 and max_iter >= 0");
  if (p->init < 0 || p->init > 2) return fail(LSOP_EINVAL, "bad init");
  int total = 0;
  for (int i = 0; i < b->count; ++i) {
    if (pcs && pcs[i] && (pcs[i]->op != b->ops[i] || !pcs[i]->built))
      return fail(LSOP_EINVAL, "preconditioner i must be built for operator i");
    total += nvec[i];
  }
  for (int k = 0; k < total; ++k) info[k] = lsop_solve_info{0, 0, INFINITY, LSOP_NOT_CONVERGED, INFINITY};
  if (b->dtype == LSOP_C64)
    st = batch_series<float>(b, pcs, reinterpret_cast<const Cx<float>* const*>(rhs_dev),
                             reinterpret_cast<Cx<float>* const*>(psi_dev), nvec, p, use_graph != 0, info, S(stream));
  else
    st = batch_series<double>(b, pcs, reinterpret_cast<const Cx<double>* const*>(rhs_dev),
                              reinterpret_cast<Cx<double>* const*>(psi_dev), nvec, p, use_graph != 0, info,
                              S(stream));
  if (st) return st;
  return overall_status(info, total);
}

int lsop_batch_info(const lsop_batch* b, int* groups, size_t* bytes) {
  if (!b) return fail(LSOP_EINVAL, "null batch");
  if (groups) *groups = (int)b->groups.size();
  if (bytes) *bytes = b->bytes;
  return LSOP_OK;
}

void lsop_batch_destroy(lsop_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  if (b->tab) (void)hipFree(b->tab);
  if (b->tmp) (void)hipFree(b->tmp);
  if (b->work) (void)hipFree(b->work);
  for (hipStream_t st : b->side) (void)hipStreamDestroy(st);
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  delete b;
}

int lsop_profile_enable(int on) {
  g_prof = on != 0;
  return LSOP_OK;
}

int lsop_profile_reset(void) {
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  return LSOP_OK;
}

static int profile_read_by(bool by_fn, lsop_kernel_stat* stats, int max_stats, int* count) {
  if (!count || (max_stats > 0 && !stats)) return fail(LSOP_EINVAL, "null argument");
  LSOP_HIP(hipDeviceSynchronize());
  std::lock_guard<std::mutex> lk(g_prof_mu);
  std::vector<lsop_kernel_stat> agg;
  for (const auto& r : g_recs) {
    float ms = 0.f;
    LSOP_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    const char* key = by_fn ? r.fn.c_str() : r.name.c_str();
    auto it = std::find_if(agg.begin(), agg.end(), [&](const lsop_kernel_stat& k) { return !strcmp(k.name, key); });
    if (it == agg.end()) {
      lsop_kernel_stat k{};
      snprintf(k.name, sizeof(k.name), "%s", key);
      agg.push_back(k);
      it = agg.end() - 1;
    }
    it->launches += 1;
    it->total_ms += ms;
    it->bytes += r.bytes;
    it->flops += r.flops;
    it->items += r.items;
  }
  *count = (int)agg.size();
  for (int i = 0; i < (int)agg.size() && i < max_stats; ++i) stats[i] = agg[i];
  return LSOP_OK;
}

int lsop_profile_read(lsop_kernel_stat* stats, int max_stats, int* count) {
  return profile_read_by(false, stats, max_stats, count);
}

int lsop_profile_read_kernels(lsop_kernel_stat* stats, int max_stats, int* count) {
  return profile_read_by(true, stats, max_stats, count);
}

int lsop_bessel_host_c(int kind, double re, double im, double* out4) {
  if (!out4) return fail(LSOP_EINVAL, "null output");
  const lsop_bessel::C z{re, im};
  if (!(re > 0) || !(im >= 0) || !std::isfinite(re) || !std::isfinite(im))
    return fail(LSOP_EINVAL, "argument must have Re z > 0 and Im z >= 0");
  if (kind == 0) {
    const lsop_bessel::C hv = lsop_bessel::hankel0_c(z);
    out4[0] = hv.re;
    out4[1] = hv.im;
    return LSOP_OK;
  }
  if (kind == 1) {
    if (lsop_bessel::c_abs(z) > 2.0) return fail(LSOP_EINVAL, "|z| must be <= 2");
    lsop_bessel::C j1, y1;
    lsop_bessel::bessel1_small_c(z, &j1, &y1);
    out4[0] = j1.re;
    out4[1] = j1.im;
    out4[2] = y1.re;
    out4[3] = y1.im;
    return LSOP_OK;
  }
  return fail(LSOP_EINVAL, "bad kind");
}

int lsop_bessel_host(int kind, double x, double* out2) {
  if (!out2 || !(x > 0)) return fail(LSOP_EINVAL, "x must be > 0");
  if (kind == 0) {
    lsop_bessel::hankel0(x, &out2[0], &out2[1]);
    return LSOP_OK;
  }
  if (kind == 1) {
    if (x > 2.0) return fail(LSOP_EINVAL, "series valid for x <= 2");
    lsop_bessel::bessel1_small(x, &out2[0], &out2[1]);
    return LSOP_OK;
  }
  return fail(LSOP_EINVAL, "bad kind");
}

}  // extern "C"
