/*
 * lsop: preconditioned Lippmann-Schwinger solver for the 2D Helmholtz equation
 * on one MI355X (gfx950).  C ABI of liblsop.so.
 *
 * Method: Eikrem, Naevdal & Jakobsen, "Iterative solution of the
 * Lippmann-Schwinger equation in strongly scattering acoustic media by
 * randomized construction of preconditioners" (arXiv 2005.01372).
 *
 * Conventions shared by every entry point
 *  - Grid: nx x nz cells of size h (metres); cell (i, j), i horizontal,
 *    j depth (j = 0 is the top row).  Vectors are stored cell-major with j
 *    fastest, n = i * nz + j (the column-wise ordering of Section 2.4).
 *  - Complex data is interleaved (re, im).  A batch of nvec vectors is
 *    [nvec][nx][nz] contiguous.  The element type of device vectors is the
 *    operator's dtype: float2 for LSOP_C64, double2 for LSOP_C128 and
 *    LSOP_MIXED.
 *  - Pointers named *_dev are device pointers (caller-owned, e.g. torch
 *    tensors), *_host are host pointers.  `stream` is a hipStream_t (NULL =
 *    default stream).  Calls enqueue work asynchronously on `stream` unless
 *    stated otherwise.
 *  - Every call returns an lsop_status.  Arguments are validated on the host
 *    before any launch; on LSOP_EINVAL / LSOP_EUNSUPPORTED outputs are left
 *    untouched.  lsop_last_error() describes the last failure of the calling
 *    thread.  No C++ exception crosses this boundary.
 *  - Device memory: by default handles own their device state (allocated at
 *    *_create, freed at *_destroy) and grow a workspace as calls need it.
 *    Callers that own all device memory instead query the sizes
 *    (lsop_state_bytes, precond_state_bytes, lsop_workspace_bytes), create
 *    handles in their own buffers (lsop_create_in, precond_create_in) and
 *    attach a workspace (lsop_attach_workspace): the operator, preconditioner
 *    and series calls then allocate no device memory.  Batches and the
 *    network keep library-owned memory.  A handle must not be used from two
 *    streams at once.
 *  - Environment (read when a handle is created; each selects between forms
 *    that compute the same result, for tests and measurements):
 *    LSOP_COL_TILE=c               column-pass tile width of new operators
 *                                  (as lsop_autotune would set it);
 *    LSOP_HODLR_LEAF_CHUNK=k       HODLR leaves inverted k at a time;
 *    LSOP_HODLR_PADDED_SAMPLING=1  HODLR sampling convolutions at the
 *                                  zero-padded period 2W on every level
 *                                  instead of the node-width period W.
 */
#ifndef LSOP_H
#define LSOP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LSOP_OK = 0,
  LSOP_EINVAL = 1,        /* bad argument (sizes, NaN/non-positive velocity, f <= 0, ...) */
  LSOP_ENOMEM = 2,        /* device allocation failed or batch exceeds capacity */
  LSOP_EHIP = 3,          /* HIP runtime error */
  LSOP_NOT_CONVERGED = 4, /* series hit max_iter; last iterate and info are written */
  LSOP_DIVERGED = 5,      /* residual non-finite or rising for 5 consecutive iterations */
  LSOP_ESINGULAR = 6,     /* I_r - W^H U is numerically singular (eq. 12) */
  LSOP_EUNSUPPORTED = 7   /* grid larger than the largest supported FFT length, bad dtype */
} lsop_status;

typedef enum { LSOP_C64 = 0, LSOP_C128 = 1, LSOP_MIXED = 2 } lsop_dtype;

/* Operator modes (x, y are [nvec][nx][nz]):
 *  LSOP_MODE_A      y = x - G0 V x            (I - G0 V of eq. 5)
 *  LSOP_MODE_G0V    y = G0 V x                (the product of Section 2.2)
 *  LSOP_MODE_AH     y = x - V^H G0^H x        (adjoint of A)
 *  LSOP_MODE_VHG0H  y = V^H G0^H x            (Alg. 2 steps 4-5, T read as conjugate transpose)
 * G0 V acts as (G0 V x)_m = sum_n K(m - n) chi_n x_n with K the integral of
 * (i/4) H0^(1)(k0 |x|) over the (equal-area disk of the) source cell, chi the
 * contrast of eq. (1).  It is evaluated by a zero-padded FFT convolution with
 * the symmetric circulant extension of the first row of G0 (Section 2.2). */
typedef enum { LSOP_MODE_A = 0, LSOP_MODE_G0V = 1, LSOP_MODE_AH = 2, LSOP_MODE_VHG0H = 3 } lsop_mode;

typedef struct lsop_op lsop_op;
typedef struct lsop_precond lsop_precond;

typedef struct {
  int nx, nz;      /* grid */
  int lx, lz;      /* FFT lengths: padded extent is 2*lx x 2*lz >= (2nx-1) x (2nz-1) */
  int dtype;       /* lsop_dtype */
  int max_vec;     /* vectors per internal batch */
  size_t state_bytes;  /* device bytes held by the handle */
  int col_tile;    /* columns per workgroup in the column FFT pass (0 = widest that fits) */
  int ny, ly;      /* 3D operators: cells and FFT length along y (1 and 0 in 2D) */
} lsop_op_info;

/* Plan an operator for an nx x nz grid and allocate its device state.
 * dtype: LSOP_C64 (complex float, FP32 accumulation), LSOP_C128 (complex
 * double) or LSOP_MIXED (complex double interface and outer residuals, with
 * complex-float inner solves; see series_solve).  max_vec bounds the
 * vectors processed per internal batch (larger calls are chunked).
 * Errors: EINVAL (nx, nz < 1, max_vec < 1), EUNSUPPORTED (nx or nz > 2048),
 * ENOMEM. */
int lsop_create(int nx, int nz, int dtype, int max_vec, lsop_op** out);

/* Set the medium (Section 2.1): contrast chi = w^2 (1/c^2 - 1/c0^2) (eq. 1),
 * the FP64 kernel table K (cell-integrated Green's function) and its
 * circulant spectrum.  vel_dev: nx*nz doubles (m/s) on the device.
 * Synchronises `stream` (to validate the velocity).  Errors: EINVAL if
 * h <= 0, freq_hz <= 0, c0 <= 0, any velocity NaN/inf/<= 0, or k0 h / sqrt(pi) > 2
 * (fewer than ~3.5 cells per background wavelength). */
int lsop_set_problem(lsop_op* op, const double* vel_dev, double h, double freq_hz, double c0,
                     void* stream);

/* The medium of the convergent Born series (Section 2.2, reviewing Osnabrugge
 * et al.): the background made dissipative, k_eps^2 = k0^2 + i eps (Re, Im
 * k_eps > 0; time factor exp(-i omega t)), and the gain put into the
 * potential, V_eps = chi - i eps r, so that the equation inside the grid is
 * unchanged: the operator becomes I - G_eps V_eps with G_eps the same
 * disk-integrated kernel at complex wavenumber (Bessel functions of complex
 * argument), and lsop_incident gives G_eps S.  Outside the grid the medium is
 * the dissipative background (absorbing).  absorb > 0 cells at the grid edges
 * form an absorbing layer: there the gain is scaled by
 * r = 1 - (1 - d / absorb) / 2 (d = cells to the edge), i.e. the medium turns
 * lossy gradually.  With eps >= max |chi| (and absorb = 0) the series with
 * H = LSOP_PC_GAMMA converges; a layer needs a larger eps (2 max |chi| was
 * measured to suffice).  vel_dev, h, freq_hz, c0 as lsop_set_problem.
 * The dissipative state (V_eps, and a [max_vec][nx][nz] temporary of the
 * widest dtype) is library-owned, allocated at the first call.  HODLR
 * preconditioners and batches reject damped operators; lsop_set_problem
 * returns the operator to the undissipated medium.  Errors: as
 * lsop_set_problem; EINVAL for eps <= 0, absorb outside [0, min(nx, nz) / 2]
 * or |k_eps h| / sqrt(pi) > 2. */
int lsop_set_problem_damped(lsop_op* op, const double* vel_dev, double h, double freq_hz, double c0, double eps,
                            int absorb, void* stream);

/* ----------------------------------------------------------------------
 * 3D operators (the extension to 3D the paper points to in Sections 1 and 4).
 * Grid nx x ny x nz cells of size h, cell (i, j, l) with l fastest:
 * n = (i ny + j) nz + l; vectors [nvec][nx][ny][nz].  G0(r) = e^{i k0 r} /
 * (4 pi r) (outgoing, exp(-i omega t)); the kernel table is its integral over
 * the ball of the cell's volume (radius a = h (3 / (4 pi))^(1/3)):
 * K = (sin k0 a - k0 a cos k0 a) / k0^3 e^{i k0 r} / r at r = h |lag| > 0 and
 * ((1 - i k0 a) e^{i k0 a} - 1) / k0^2 on the diagonal; (G0 V)_{mn} =
 * K(m - n) chi_n.  The FFT convolution runs in five passes (z rows, y columns
 * per x-plane, x columns with the spectrum, y columns back, z rows back with
 * the epilogue) on an intermediate of nx * 2ly * 2lz values per vector.
 * lsop_apply, lsop_residual, lsop_apply_noalloc, series_solve, gmres_solve and
 * the LOWRANK / SCALAR preconditioners take 3D operators unchanged; HODLR,
 * batches, the dissipative medium and the network are 2D only.  3D operators
 * are library-owned (no lsop_create_in form). */
int lsop_create3d(int nx, int ny, int nz, int dtype, int max_vec, lsop_op** out);
/* Contrast (eq. 1), kernel table and spectrum; vel_dev nx*ny*nz doubles.  Errors as lsop_set_problem
 * (k0 a > 2: grid too coarse). */
int lsop_set_problem3d(lsop_op* op, const double* vel_dev, double h, double freq_hz, double c0, void* stream);
/* psi0 of point sources: src_ijl_host[3 k + {0, 1, 2}] = (i, j, l), density amp / h^3. */
int lsop_incident3d(lsop_op* op, const int* src_ijl_host, const double* amp_reim_host, int nsrc, void* psi0_dev,
                    void* stream);

/* y = op(x) for nvec vectors (mode: lsop_mode).  x and y may alias. */
int lsop_apply(lsop_op* op, int mode, const void* x_dev, void* y_dev, int nvec, void* stream);

/* r = A psi - rhs and, if rnorm2_dev != NULL, rnorm2_dev[k] = ||r_k||_2^2
 * (double, overwritten).  Any of psi, rhs, r may alias.  (Eq. 13.) */
int lsop_residual(lsop_op* op, const void* psi_dev, const void* rhs_dev, void* r_dev,
                  double* rnorm2_dev, int nvec, void* stream);

/* Incident fields of point sources (Section 2.1 source representation): a
 * source of amplitude amp in cell s has density amp / h^2 in that cell, so
 * psi0_m = amp * K(m - s) / h^2.  src_i, src_j: nsrc cell indices (host);
 * amp_reim: 2*nsrc doubles (re, im) or NULL for unit amplitudes.
 * psi0_dev: [nsrc][nx][nz].  Errors: EINVAL for a source outside the grid. */
int lsop_incident(lsop_op* op, const int* src_i_host, const int* src_j_host,
                  const double* amp_reim_host, int nsrc, void* psi0_dev, void* stream);

/* Autotune the FFT tile shape for batches of nvec vectors: times the
 * column-pass kernel for each supported tile width (16, 8, 4, 2 columns per
 * workgroup) on this operator's grid with HIP events and keeps the fastest for
 * later calls.  Requires lsop_set_problem.  Synchronises `stream`; overwrites
 * the operator's internal intermediate buffer only. */
int lsop_autotune(lsop_op* op, int nvec, void* stream);

/* Copy the FP64 kernel table K[p][q] (p < nx, q < nz; complex double,
 * [nx][nz]) to table_dev.  Diagnostic. */
int lsop_kernel_table(const lsop_op* op, void* table_dev, void* stream);

int lsop_info(const lsop_op* op, lsop_op_info* info);
void lsop_destroy(lsop_op* op);

/* Caller-owned memory.  lsop_state_bytes: device bytes of an operator's state
 * (contrast, FP64 kernel table, circulant spectrum, twiddles, the FFT
 * intermediate of max_vec vectors, source staging) for lsop_create's
 * arguments; host only, no device call.  Errors as lsop_create. */
int lsop_state_bytes(int nx, int nz, int dtype, int max_vec, size_t* bytes);

/* lsop_create with the state carved from the caller's device buffer state_dev
 * of state_bytes bytes (256-byte aligned, at least lsop_state_bytes; it must
 * outlive the handle, and lsop_destroy does not free it).  Errors: as
 * lsop_create; ENOMEM if state_bytes is too small; EINVAL if state_dev is
 * NULL or not 256-byte aligned. */
int lsop_create_in(int nx, int nz, int dtype, int max_vec, void* state_dev, size_t state_bytes, lsop_op** out);

/* Device workspace that lsop_set_problem and series_solve on nvec right-hand
 * sides with start `init` (lsop_init) need; host only. */
int lsop_workspace_bytes(const lsop_op* op, int nvec, int init, size_t* bytes);

/* Hand the operator a caller-owned workspace (ws_dev, ws_bytes; 256-byte
 * aligned; it must outlive the handle or a later attach).  From then on
 * lsop_set_problem, series_solve and the builds of this operator's
 * preconditioners take their temporaries from it and never allocate; a call
 * that needs more fails with ENOMEM before any launch.  Replaces any
 * library-owned workspace (freed after a device synchronisation).  ws_dev =
 * NULL returns the operator to library-owned growth. */
int lsop_attach_workspace(lsop_op* op, void* ws_dev, size_t ws_bytes);

/* Diagnostic: device allocations (hipMalloc / hipMallocAsync calls) the
 * library has made in this process. */
int lsop_alloc_count(size_t* calls);

/* lsop_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same passes, with the FFT intermediate in a fixed 64 MiB device array of the
 * library (allocated with the library's code object on each GPU it runs on and
 * held until the process ends) instead of the operator's buffer, processed in
 * chunks of as many vectors as fit.  Makes no device allocation.  Errors: as
 * lsop_apply; EINVAL if one vector's intermediate (nx * 2 lz complex values of
 * the operator's widest dtype) exceeds 64 MiB.  All calls on one GPU share the
 * array: calls that overlap on one GPU (several streams or threads) race. */
int lsop_apply_noalloc(lsop_op* op, int mode, const void* x_dev, void* y_dev, int nvec, void* stream);
const char* lsop_last_error(void);

/* ----------------------------------------------------------------------
 * Preconditioners H for the series of eq. (11).
 *  LSOP_PC_IDENTITY  H = I (the Born series, Section 2.2).
 *  LSOP_PC_SCALAR    H = alpha I (Section 2.2: the scalar choice of the
 *                    homotopy series, alpha < 1).
 *  LSOP_PC_GAMMA     H = gamma = i V_eps / eps pointwise, for an operator set
 *                    by lsop_set_problem_damped: the series is then the
 *                    convergent Born series (Section 2.2), started from
 *                    gamma psi0 (LSOP_INIT_H_RHS).  Holds no state; reads the
 *                    operator's current V_eps and eps at every apply.
 *  LSOP_PC_LOWRANK   H = I + U Z W^H with G0 V ~= U W^H from the randomized
 *                    range finder of Alg. 2 (power_iters = q) and
 *                    Z = (I_r - W^H U)^{-1} by Sherman-Morrison-Woodbury
 *                    (eq. 12).  `rank` + `oversample` probe vectors; with
 *                    oversample p > 0 the (rank + p)-column factorisation is
 *                    truncated to `rank` columns through an FP64 SVD of its
 *                    (rank + p) x (rank + p) core (W~ = Q2 R2, R2^H =
 *                    U_b S V_b^H, U = Q U_b S restricted to the leading
 *                    `rank` singular values, W = Q2 V_b likewise; Halko et
 *                    al. 2011, Section 5; the paper uses p = 0).
 *  LSOP_PC_HODLR     H = A_h^{-1}, A_h the hierarchically off-diagonal
 *                    low-rank approximation of A = I - G0 V (Section 2.4,
 *                    Fig. 1): cells in column-wise order, a binary tree of
 *                    `levels` levels of vertical strips (node of level l:
 *                    nx / 2^l grid columns, split into equal halves), dense
 *                    diagonal leaves of nx / 2^levels columns, and both
 *                    off-diagonal blocks of every node approximated by Alg. 1
 *                    (q = power_iters, 0 in the paper) with `rank` probes,
 *                    the block products done as
 *                    FFT convolutions on the node's sub-domain.  A_h is
 *                    inverted exactly, level by level, by Sherman-Morrison-
 *                    Woodbury on the off-diagonal factors (the 2 x 2 block
 *                    inverse of Section 2.4 kept in factored form, with no
 *                    recompression); the leaves by the recursive 2 x 2 block
 *                    formula, in FP32 for complex-FP32 operators (including
 *                    the mixed mode) and FP64 for complex-FP64 ones; the node
 *                    cores always inverted in FP64 and applied in the
 *                    operator's precision.  Requires nx divisible by 2^levels,
 *                    (nx / 2^levels) * nz a multiple of 64 and at most 8192.
 * ---------------------------------------------------------------------- */
typedef enum {
  LSOP_PC_IDENTITY = 0,
  LSOP_PC_LOWRANK = 1,
  LSOP_PC_HODLR = 2,
  LSOP_PC_SCALAR = 3,
  LSOP_PC_GAMMA = 4
} lsop_pc_kind;

typedef struct {
  int kind;         /* lsop_pc_kind */
  int rank;         /* LOWRANK: kept rank r; HODLR: probes per block; 1 <= rank <= 256 */
  int power_iters;  /* q >= 0 (Alg. 1 power iterations; the paper's HODLR uses q = 0) */
  uint64_t seed;    /* Philox4x32-10 key when no probe block is supplied */
  int levels;       /* HODLR tree depth, >= 1 (ignored otherwise) */
  int oversample;   /* LOWRANK: extra probes p >= 0, rank + p <= 256 (0 elsewhere) */
  double alpha;     /* SCALAR: H = alpha I, alpha finite and non-zero */
  int q_from_level; /* HODLR: the power iterations run on tree levels >= this one only (0: every level; the
                       wide blocks of the top levels were measured to need none at 1024^2, the narrow deep
                       ones do); >= 0, ignored elsewhere */
  int min_width;    /* HODLR: the other stopping rule of Section 2.4, a minimum size: no split leaves a node
                       narrower than min_width grid columns, so the tree depth is the smaller of `levels` and
                       the deepest level whose nodes are at least min_width wide (0 or 1: no limit; >= 0);
                       precond_depth reports the depth taken */
} lsop_precond_params;

/* Allocate a preconditioner for `op` (U, W: rank x n complex in the inner
 * dtype of op; Z: rank x rank).  Errors: EINVAL, ENOMEM. */
int precond_create(lsop_op* op, const lsop_precond_params* params, lsop_precond** out);

/* Caller-owned memory: device bytes of the preconditioner's state (*state)
 * and of the transient workspace its build needs (*build_ws; it comes from
 * the operator's attached workspace, so attach at least the larger of this
 * and lsop_workspace_bytes).  Host only. */
int precond_state_bytes(const lsop_op* op, const lsop_precond_params* params, size_t* state, size_t* build_ws);

/* precond_create with the state carved from the caller's buffer (256-byte
 * aligned, at least precond_state_bytes' *state; it must outlive the handle,
 * precond_destroy does not free it).  Errors: as precond_create; ENOMEM if
 * state_bytes is too small. */
int precond_create_in(lsop_op* op, const lsop_precond_params* params, void* state_dev, size_t state_bytes,
                      lsop_precond** out);

/* Build H (Alg. 2 then eq. 12).  omega_dev: (rank + oversample) x nx*nz real
 * doubles, probe k contiguous, or NULL to draw standard normals on the device with
 * Philox4x32-10 (counter = (pair index lo, hi, k, 0), key = seed) and
 * Box-Muller.  Columns of the range basis that are numerically dependent are
 * dropped (zero columns of U), so chi = 0 gives H = I exactly.  Synchronises
 * `stream`.  Errors: ESINGULAR if I - W^H U is singular.
 * HODLR: omega_dev holds levels * rank probes (or Philox probes k = l * rank
 * .. (l + 1) * rank - 1 for tree level l); the probes of level l restricted to
 * the cells of a node's second half sample its upper off-diagonal block, to
 * the first half its lower block.  Each half's samples are orthonormalised
 * separately (Cholesky-QR twice, FP64 small factors).  Errors: ESINGULAR if a
 * leaf block or a node's Woodbury core is singular. */
int precond_build(lsop_precond* pc, const void* omega_dev, void* stream);

/* Builds `count` preconditioners (Philox probes, as precond_build with
 * omega_dev = NULL) concurrently: `streams` (1..16) host threads, each with a
 * non-blocking stream of its own, take the preconditioners one at a time,
 * largest grid first.  Independent builds of small grids leave most of the
 * device idle alone (the instances of an uneven batch, Section 3.1.2's many
 * media); running several at once fills it.  The preconditioners must belong
 * to distinct operators (EINVAL otherwise: an operator's scratch is shared by
 * its builds).  Synchronises the device before and all its streams after;
 * returns the first failure of any build (the others still complete). */
int precond_build_batch(lsop_precond* const* pcs, int count, int streams);

/* y = H x for nvec vectors (x, y in the inner dtype of the op). */
int precond_apply(lsop_precond* pc, const void* x_dev, void* y_dev, int nvec, void* stream);

/* rank kept, compression 2 r / n (Section 3.1.1), device bytes held.
 * HODLR: rank = r, compression = stored complex entries / n^2. */
int precond_info(const lsop_precond* pc, int* rank, double* compression, size_t* bytes);
/* Depth of a HODLR preconditioner's tree after the min_width rule (the number of probe blocks precond_build
 * takes); 0 for the other kinds.  Host only. */
int precond_depth(const lsop_precond* pc, int* levels);
void precond_destroy(lsop_precond* pc);

/* ----------------------------------------------------------------------
 * The preconditioned scattering series (eqs. 10-11, 13-14).
 *   psi_0 = H psi0 (init = LSOP_INIT_H_RHS, the paper's phi_0), or psi_dev
 *   as given (LSOP_INIT_USER), or 0 (LSOP_INIT_ZERO), or, per right-hand
 *   side, whichever of psi_dev (a candidate such as a learned warm start) and
 *   H psi0 has the smaller residual (LSOP_INIT_BEST; the candidate is also
 *   replaced when its residual is not finite; LSOP_MIXED treats it as USER);
 *   repeat: a = A psi - psi0 (eq. 13); stop when ||a|| / ||psi0|| <= tol;
 *           psi <- psi - H a (eq. 11; eq. 14 read as psi - (a + U Z W^H a)).
 * Each right-hand side stops on its own; the returned iterate is the one whose
 * residual passed.  Cap max_iter (default 30, Section 3.1).  DIVERGED if the
 * residual is non-finite or rises 5 times in a row.
 * LSOP_MIXED operators run iterative refinement: outer residuals and the
 * accumulated solution in complex double, inner series in complex float to
 * inner_tol, until the FP64 relative residual <= tol (at most refine_max
 * outer steps).  pc may be NULL (Born series).  Synchronises `stream` once
 * per iteration (convergence test on the host).
 * rhs_dev, psi_dev: [nvec][nx][nz]; info_host: nvec entries.  Returns OK if
 * every right-hand side converged, else the first failing status. */
typedef enum { LSOP_INIT_H_RHS = 0, LSOP_INIT_ZERO = 1, LSOP_INIT_USER = 2, LSOP_INIT_BEST = 3 } lsop_init;

typedef struct {
  double tol;        /* relative residual target */
  int max_iter;      /* per series (inner series for MIXED) */
  int init;          /* lsop_init */
  int refine_max;    /* MIXED only: outer refinement steps (default 8) */
  double inner_tol;  /* MIXED only: inner relative tolerance (default 1e-5) */
} lsop_solve_params;

typedef struct {
  int iters;            /* series updates performed (summed over refinement steps) */
  int refine_steps;     /* outer steps (MIXED) */
  double rel_residual;  /* ||A psi - psi0|| / ||psi0|| of the returned iterate */
  int status;           /* lsop_status of this right-hand side */
  double rel_residual0; /* relative residual of the initial iterate (first series for MIXED) */
} lsop_solve_info;

int series_solve(lsop_op* op, lsop_precond* pc, const void* rhs_dev, void* psi_dev, int nvec,
                 const lsop_solve_params* params, lsop_solve_info* info_host, void* stream);

/* series_solve from point sources (Section 2.1: the wavefield of given sources, the paper's problem
 * statement): the incident fields of lsop_incident (src_i_host, src_j_host, amp_reim_host as there) are formed
 * in the operator's workspace and solved for; psi_dev: [nsrc][nx][nz] output (input with LSOP_INIT_USER /
 * LSOP_INIT_BEST); info_host: nsrc entries.  The same results as lsop_incident followed by series_solve.
 * Workspace: series_sources_workspace_bytes (the nsrc incident fields ahead of series_solve's own); grown by
 * the library or taken from the attached workspace.  2D operators.  Errors: as lsop_incident and
 * series_solve. */
int series_solve_sources(lsop_op* op, lsop_precond* pc, const int* src_i_host, const int* src_j_host,
                         const double* amp_reim_host, int nsrc, void* psi_dev, const lsop_solve_params* params,
                         lsop_solve_info* info_host, void* stream);
int series_sources_workspace_bytes(const lsop_op* op, int nsrc, int init, size_t* bytes);

/* ----------------------------------------------------------------------
 * Restarted GMRES(m), the Krylov method the paper compares the preconditioned
 * series with (Section 3.2.3), right-preconditioned by H: it solves
 * A H y = psi0 - A psi_start and returns psi = psi_start + H y, so it
 * converges whatever the spectral radius of M = I - H A (the series needs
 * rho(M) < 1).  Every right-hand side runs its own Arnoldi process (classical
 * Gram-Schmidt applied twice, FP64 sums), in lockstep with the others; the
 * Hessenberg least-squares problems are solved on the host in FP64 (Givens
 * rotations).  A cycle of a right-hand side ends when its residual estimate
 * reaches tol, after `restart` iterations, at max_iter or on breakdown; the
 * true residual ||A psi - psi0|| / ||psi0|| then decides convergence.
 * info[v].iters counts inner iterations (one A and one H application each).
 * pc NULL or identity: unpreconditioned.  LSOP_MIXED operators run FP64
 * iterative refinement around complex-FP32 GMRES (inner_tol, refine_max as in
 * series_solve).  Workspace: gmres_workspace_bytes ((restart + 3) vectors per
 * right-hand side plus small terms); grown by the library or taken from the
 * attached workspace.  Synchronises `stream` once per inner iteration.
 * Returns OK if every right-hand side converged, else the first failing
 * status (NOT_CONVERGED at max_iter). */
typedef struct {
  double tol;        /* relative residual target */
  int restart;       /* Krylov dimension per cycle, 1..200 */
  int max_iter;      /* inner iterations in total (per refinement step for MIXED) */
  int init;          /* LSOP_INIT_H_RHS, LSOP_INIT_ZERO or LSOP_INIT_USER */
  int refine_max;    /* MIXED only: outer refinement steps (default 8) */
  double inner_tol;  /* MIXED only: inner relative tolerance (default 1e-5) */
} lsop_gmres_params;

int gmres_solve(lsop_op* op, lsop_precond* pc, const void* rhs_dev, void* psi_dev, int nvec,
                const lsop_gmres_params* params, lsop_solve_info* info_host, void* stream);
int gmres_workspace_bytes(const lsop_op* op, int nvec, int restart, size_t* bytes);

/* ----------------------------------------------------------------------
 * Frequency sweep (Section 3.1): the problem at each of nfreq increasing
 * frequencies (the paper sweeps integer frequencies lowest first), the
 * series of eq. (11) with a preconditioner of kind pc0->kind built per
 * frequency, the rank managed as in Section 3.1: the series gets at most
 * max_iter iterations (30 in the paper); if a frequency does not converge,
 * its preconditioner is rebuilt with rank + rank_step and the series
 * restarted from H psi0 (at most max_rebuilds times); if it converged but
 * needed more than escalate_above iterations (10 in the paper), the next
 * frequency starts at rank + rank_step (the paper's steps: +200 for the
 * simple preconditioner, +5 for the hierarchical one).  Sources are point
 * sources (as lsop_incident) with amplitude 1, or, with ricker_fc > 0, the
 * spectrum of a Ricker wavelet of centre frequency ricker_fc delayed by
 * 1 / ricker_fc: (2 / sqrt(pi)) f^2 / fc^3 exp(-f^2 / fc^2) exp(-2 pi i f / fc)
 * (the paper's source; its normalisation is not stated).
 * psi_dev: [nfreq][nsrc][nx][nz] in the operator's dtype (also scratch for the
 * next frequency's incident fields).  info_host[k]: the frequency's final
 * rank, rebuilds, largest iteration count and residual, status.  The
 * operator's medium is left at the last frequency.  Synchronous.  Returns OK
 * if every frequency converged, else the first failing status. */
typedef struct {
  double tol;          /* relative residual per source */
  int max_iter;        /* series iterations per attempt (30) */
  int escalate_above;  /* raise the rank for the next frequency above this many iterations (10) */
  int rank_step;       /* rank increase (200 simple, 5 HODLR in the paper) */
  int rank_max;        /* cap (<= 256; 0: 256) */
  int max_rebuilds;    /* rebuilds per frequency */
  double ricker_fc;    /* Hz; 0: unit amplitudes */
} lsop_sweep_params;

typedef struct {
  double freq;
  int rank;               /* rank of the preconditioner that produced the returned fields */
  int rebuilds;           /* rebuilds at this frequency */
  int iters_max;          /* largest iteration count over the sources */
  int status;             /* lsop_status of the frequency */
  double rel_residual_max;
} lsop_sweep_info;

int lsop_sweep(lsop_op* op, const double* vel_dev, double h, double c0, const double* freqs_host, int nfreq,
               const lsop_precond_params* pc0, const lsop_sweep_params* params, const int* src_i_host,
               const int* src_j_host, int nsrc, void* psi_dev, lsop_sweep_info* info_host, void* stream);

/* ----------------------------------------------------------------------
 * Batches of problems of uneven size (many instances of Section 2's problem,
 * each with its own grid, medium, frequency and sources).  A batch wraps
 * existing operator handles (created and set up by the caller, all complex
 * float or all complex double; they must outlive the batch) and groups the
 * instances by grid shape.  Every FFT pass of the LS operator (Section 2.2)
 * is then one launch per shape group over all vectors of all its members,
 * each vector carrying its own instance's contrast and spectrum.
 * ---------------------------------------------------------------------- */
typedef struct lsop_batch lsop_batch;

/* Errors: EINVAL (null / unset operators, mixed dtypes), EUNSUPPORTED (LSOP_MIXED). */
int lsop_batch_create(int count, lsop_op* const* ops, lsop_batch** out);

/* y_i = op_i(x_i) (mode as lsop_apply) for nvec[i] vectors of instance i;
 * x_dev[i], y_dev[i]: [nvec[i]][nx_i][nz_i] device buffers (no aliasing).
 * Synchronises `stream` once to stage the per-vector operand tables. */
int lsop_batch_apply(lsop_batch* b, int mode, const void* const* x_dev, void* const* y_dev, const int* nvec,
                     void* stream);

/* Column-pass tile width per shape group, timed once per (dtype, shape,
 * vector-count class) in the process and reused by later batches. */
int lsop_batch_autotune(lsop_batch* b, void* stream);

/* The series of eq. (11) for every vector of every instance, advanced in
 * lockstep: each iteration is one preconditioner update per instance
 * (pcs[i], NULL or identity: Born) and one grouped residual evaluation.
 * Vectors that finish (stopping rule of series_solve) are frozen: their
 * residual is zeroed before the update, so their psi keeps the iterate whose
 * residual was evaluated.  use_graph != 0: after the first iteration the
 * launch sequence of one iteration is captured once as a HIP graph (on a
 * stream of the library's own; no memset nodes) and replayed.  info: one
 * entry per vector, instance by instance.  Synchronous.  Returns OK if every
 * vector converged, else the first failing status; init as in series_solve
 * (LSOP_INIT_USER: psi holds the start). */
int lsop_batch_solve(lsop_batch* b, lsop_precond* const* pcs, const void* const* rhs_dev, void* const* psi_dev,
                     const int* nvec, const lsop_solve_params* params, int use_graph, lsop_solve_info* info,
                     void* stream);

/* number of shape groups and device bytes held by the batch (tables, intermediates, work) */
int lsop_batch_info(const lsop_batch* b, int* groups, size_t* bytes);
void lsop_batch_destroy(lsop_batch* b);

/* ----------------------------------------------------------------------
 * Learned warm start (a convolutional network giving phi_0 of the series;
 * Section 2.2: the fixed point of eq. 11 does not depend on phi_0).
 * U-Net with `levels` resolutions (channels base * 2^l), two 3x3 convolutions
 * + ReLU per level, 2x2 average pooling, nearest 2x upsampling with
 * concatenation [upsampled, skip], and a 1x1 head.  Activations FP32
 * [B][H][W][C] (channels fastest); convolutions run on bf16 matrix cores with
 * FP32 accumulation; FP32 master weights, trained with Adam on the mean
 * squared error.  Parameters are flat FP32, layer by layer (e0a, e0b, ...,
 * e(L-1)b, d(L-2)a, d(L-2)b, ..., d0b, head), each as weights
 * [kh][kw][Ci][Co] followed by Co biases.  H and W must be multiples of
 * 2^(levels-1) and within the sizes given at creation.  Not thread-safe;
 * all calls are asynchronous on `stream` unless noted.
 * ---------------------------------------------------------------------- */
typedef struct unet unet;

int unet_create(int levels, int base, int cin, int cout, int max_batch, int max_h, int max_w, unet** out);
int unet_param_count(const unet* u, size_t* n);
/* Loads FP32 parameters (device) and resets the optimizer state. */
int unet_set_params(unet* u, const float* params_dev, void* stream);
/* He-normal initialisation (weights N(0, 2 / fan_in) with fan_in = k^2 Ci,
 * biases 0; the normal draws come from the device Philox4x32-10 stream with
 * key `seed`), and resets the optimizer state.  The paper leaves the start
 * free; this is the usual start for ReLU networks. */
int unet_init_params(unet* u, unsigned long long seed, void* stream);
int unet_get_params(const unet* u, float* params_dev, void* stream);
/* y = net(x): x [B][H][W][cin], y [B][H][W][cout] (device FP32).  x must stay
 * valid until a following unet_backward. */
int unet_forward(unet* u, const float* x_dev, int B, int H, int W, float* y_dev, void* stream);
/* Parameter gradients for the output gradient dy of the last forward pass. */
int unet_backward(unet* u, const float* dy_dev, void* stream);
int unet_get_grads(const unet* u, float* grads_dev, void* stream);
/* Forward, mean squared error against target, backward, one Adam step
 * (beta 0.9 / 0.999, eps 1e-8) at rate lr.  loss_host (optional) receives the
 * loss; the call then synchronises `stream`. */
int unet_train_step(unet* u, const float* x_dev, const float* target_dev, int B, int H, int W, float lr,
                    double* loss_host, void* stream);
/* Network inputs for nvec incident fields of `op` (complex float for
 * LSOP_C64 operators, complex double otherwise):
 * per cell [c/c0 - 1, Re psi0 / s_v, Im psi0 / s_v, k0 h], s_v the RMS of
 * field v; x_dev [nvec][nx][nz][4], scale_dev [nvec] receives s_v. */
int unet_pack_inputs(unet* u, const lsop_op* op, const void* psi0_dev, int nvec, float* x_dev, float* scale_dev,
                     void* stream);
/* Training target of solution psi for incident field psi0: the scaled
 * scattered field ((psi - psi0) / s_v) as (re, im), t_dev [nvec][nx][nz][2];
 * scale_dev as returned by unet_pack_inputs. */
int unet_pack_target(const lsop_op* op, const void* psi_dev, const void* psi0_dev, const float* scale_dev, int nvec,
                     float* t_dev, void* stream);
/* phi_0 = psi0 + s_v net(inputs) for nvec incident fields (the network is
 * trained on the scaled scattered field (psi - psi0) / s_v); psi_dev
 * [nvec][nx][nz] in the dtype of psi0. */
int unet_warm_start(unet* u, const lsop_op* op, const void* psi0_dev, void* psi_dev, int nvec, void* stream);
int unet_info(const unet* u, size_t* params, size_t* bytes);
void unet_destroy(unet* u);

/* Diagnostics: FP64 Bessel evaluations used for the kernel table, on the host
 * (kind 0: (J0, Y0) at x > 0; kind 1: (J1, Y1) at 0 < x <= 2). */
int lsop_bessel_host(int kind, double x, double* out2);
/* The same at complex argument z = re + i im (Re z > 0, Im z >= 0), as used for
 * the dissipative kernel table: kind 0: H0^(1)(z) as (re, im) in out4[0..1];
 * kind 1: J1(z), Y1(z) for |z| <= 2 as out4[0..3]. */
int lsop_bessel_host_c(int kind, double re, double im, double* out4);

/* Per-kernel timing (diagnostics).  While enabled, every kernel launch of the
 * library is bracketed by HIP events recorded on its launch stream, and the
 * kernel's algorithmic HBM bytes (compulsory reads + writes of that launch,
 * by the formulas documented with each kernel) are accumulated by name.
 * lsop_profile_read synchronises the device and returns up to max_stats
 * entries (count = number of distinct kernels).  Not thread-safe. */
typedef struct {
  char name[48];
  int launches;
  double total_ms;      /* sum of event-measured launch durations */
  double bytes;         /* sum of algorithmic bytes */
  double flops;         /* sum of algorithmic floating-point operations */
  double items;         /* vectors processed (FFT passes) or output columns (GEMMs) */
} lsop_kernel_stat;

int lsop_profile_enable(int on);
int lsop_profile_reset(void);
/* aggregated by use (e.g. "lsop_cols": the column pass of the LS operator) */
int lsop_profile_read(lsop_kernel_stat* stats, int max_stats, int* count);
/* aggregated by kernel function, named as rocprofv3 names it without the
 * namespace and argument list (e.g. "k_cols<float, 1024, 8>") */
int lsop_profile_read_kernels(lsop_kernel_stat* stats, int max_stats, int* count);

#ifdef __cplusplus
}
#endif
#endif /* LSOP_H */
