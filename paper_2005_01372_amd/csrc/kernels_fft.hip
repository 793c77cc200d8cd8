// FFT-convolution kernels of the LS operator (Section 2.2) and its set-up
// (contrast of eq. 1, cell-integrated kernel table, circulant spectrum).
//
// The product G0 V x is a linear convolution of the nx x nz grid with the
// lag table K, evaluated as a circular convolution on the padded 2 lx x 2 lz
// array (lx >= nx, lz >= nz).  Because the input occupies only the first
// half of each padded axis, a length-2L transform splits into two length-L
// transforms:
//   X[2m]   = FFT_L(u)[m],       X[2m+1] = FFT_L(u . w_{2L}^n)[m],
// and because only the first half of the output is kept, the inverse is
//   y[n] = IFFT_L(Y_even)[n] + w_{2L}^{-n} IFFT_L(Y_odd)[n].
// Three passes over HBM implement one application:
//   1. rows (fixed i, j contiguous): u = chi . x (or x), two FFTs -> tmp[i][0..2lz)
//   2. columns of tmp (fixed c, i strided): both x-halves: FFT, multiply by
//      the spectrum, inverse FFT, recombine -> tmp (only rows i < nx kept)
//   3. rows: two inverse FFTs, recombine, crop to j < nz, epilogue
//      (x - conv, conv, x - chi conv, chi conv; optional residual and norm).
// The spectrum gs[h][c][m] holds F(K~)[2m + h][kz(c)] / (px pz) with the
// column index c in the split order of pass 1 (kz(c) = 2 (c mod lz) + c / lz).
#include "fft_engine.hpp"
#include "bessel.hpp"
#include "internal.hpp"

namespace lsop {

int fft_length_for(int n) {
  static const int lens[] = {32, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 2048};
  for (int L : lens)
    if (L >= n) return L;
  return -1;
}

int fft_length_sub(int n) {
  static const int lens[] = {2, 4, 8, 16};
  for (int L : lens)
    if (L >= n) return L;
  return fft_length_for(n);
}

// Threads per workgroup of the row kernels: 256 unless the groups' two
// exchange buffers plus the twiddle table would not fit in 144 KiB of LDS.
template <typename T, int L>
constexpr int rows_threads() {
  int t = 256;
  while (t > FftPlan<L>::G &&
         (t / FftPlan<L>::G) * 2 * lds_len<L>() * (int)sizeof(Cx<T>) + lds_len<L>() * (int)sizeof(Cx<T>) >
             144 * 1024)
    t /= 2;
  return t;
}

// ------------------------------------------------------------------ pass 1
// One group per row; the even and odd halves are transformed together
// (fft2_regs), and the next row's input is prefetched into registers while
// the current row is transformed.
//
// Sub-domain batches: with nodes > 1 every stored vector of nodes * nx rows is
// treated as `nodes` independent nx-row strips (slot = vector * nodes + node),
// each with its own slice of chi; rows i outside [lo, hi) of a strip read as
// zero (pass 1) or are not written (pass 3).
//
// Grouped batches (tab != NULL): slot s is one vector of one of several
// operators of the same shape; tab[s] holds its operands (vector, contrast,
// spectrum, right-hand side, norm accumulator).
template <typename T, int L>
__global__ __launch_bounds__((rows_threads<T, L>())) void k_rows_fwd(const Cx<T>* __restrict__ x,
                                                                     const T* __restrict__ chi,
                                                                     Cx<T>* __restrict__ tmp,
                                                                     const int* __restrict__ vidx, int nx, int nz,
                                                                     int nitems, int mulchi,
                                                                     const Cx<T>* __restrict__ tw2, int nodes, int lo,
                                                                     int hi, const Slot<T>* __restrict__ tab,
                                                                     int trows, RowMap rm) {
  using P = FftPlan<L>;
  constexpr int G = P::G, E = P::E, GPW = rows_threads<T, L>() / G;
  __shared__ Cx<T> sbuf[GPW][2][lds_len<L>()];
  __shared__ Cx<T> stw[lds_len<L>()];
  stage_twiddles<T, L>(stw, tw2);
  __syncthreads();
  const int grp = threadIdx.x / G, g = threadIdx.x % G;
  const size_t vstride = (size_t)nodes * nx * nz;
  const int step = gridDim.x * GPW;
  Cx<T> px[E];
  T pc[E];
  auto fetch = [&](int base) {
    const int item = base + grp;
    const int it = item < nitems ? item : nitems - 1;
    const int slot = it / rm.ns, i = rm.xa + rm.xs * (it % rm.ns);
    const int node = slot % nodes, vs = slot / nodes;
    const int vi = vidx ? vidx[vs] : vs;
    const size_t row = (size_t)node * nx + i;
    const Cx<T>* xr = tab ? tab[slot].x + row * nz : x + (size_t)vi * vstride + row * nz;
    const T* cr = (tab ? tab[slot].chi : chi) + row * nz;
    const bool in = i >= lo && i < hi;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = fft_elem<L>(g, e);
      px[e] = (in && p < nz) ? xr[p] : czero<T>();
      pc[e] = (mulchi && in && p < nz) ? cr[p] : T(1);
    }
  };
  int base = blockIdx.x * GPW;
  if (base < nitems) fetch(base);
  for (; base < nitems; base += step) {
    const int item = base + grp;
    const bool valid = item < nitems;
    const int it = valid ? item : nitems - 1;
    const int slot = it / rm.ns, ii = it % rm.ns;
    Cx<T> a[E], b[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = fft_elem<L>(g, e);
      a[e] = pc[e] * px[e];
      b[e] = a[e] * tw_lo<T, L>(stw, p);
    }
    if (base + step < nitems) fetch(base + step);
    Cx<T>* tr = tmp + ((size_t)slot * trows + ii) * (2 * L);
    fft2_regs<T, L, false>(a, b, g, sbuf[grp][0], sbuf[grp][1], stw);
    if (valid) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int p = fft_elem<L>(g, e);
        tr[p] = a[e];
        tr[L + p] = b[e];
      }
    }
    wave_sync();
  }
}

// ------------------------------------------------------------------ pass 2
// A workgroup owns C adjacent columns of tmp (C * sizeof(Cx<T>) contiguous
// bytes per row) and one wavefront group per column.  The tile is staged in
// LDS column-major with an odd column stride (conflict-free transposition);
// each column's LDS slot then serves as one of the two exchange buffers of
// that group's interleaved even/odd FFT pair, xbuf as the other.
template <typename T, int L>
struct ColTile {
  // widest tile that keeps 128-byte row segments and fits the LDS and thread budgets; transforms done by a
  // single lane (lengths 2-8: the x-transforms of narrow sub-domains) take 256-column tiles, so that
  // workgroups are not mostly empty and their number does not swamp the dispatcher (measured: wider tiles for
  // the multi-lane lengths 16-64 were slightly slower)
  static constexpr int stride = lds_len<L>() + 1;
  static constexpr int lds_cap =
      (156 * 1024 - lds_len<L>() * (int)sizeof(Cx<T>)) / ((stride + lds_len<L>()) * (int)sizeof(Cx<T>));
  static constexpr int line = 128 / (int)sizeof(Cx<T>);
  static constexpr int wide = FftPlan<L>::G == 1 ? 256 : 1;
  static constexpr int want = line > wide ? line : wide;
  static constexpr int c0 = want < lds_cap ? want : lds_cap;
  static constexpr int thr_cap = 1024 / FftPlan<L>::G;
  static constexpr int c1 = c0 < thr_cap ? c0 : thr_cap;
  static constexpr int C = c1 >= 256 ? 256 : c1 >= 128 ? 128 : c1 >= 64 ? 64 : c1 >= 32 ? 32 : c1 >= 16 ? 16
                         : c1 >= 8   ? 8   : c1 >= 4   ? 4   : c1 >= 2  ? 2  : 1;
};

// blockIdx -> logical id so that consecutive logical ids run on the same XCD
// (workgroups are dispatched round-robin over the 8 XCDs).
__device__ __forceinline__ int xcd_logical_block(int b, int nb) {
  const int per = nb / 8, rem = nb % 8, x = b % 8;
  return x * per + (x < rem ? x : rem) + b / 8;
}

// Tile transfers between rows of global memory (row stride pz) and a column-major LDS tile (column stride lst,
// rows padded by lds_pad): n rows, of which rows i >= nrow read as zero (tile_in) or are not written (tile_out).
// Complex-float tiles of even width move two adjacent columns per 16-byte access, half the memory instructions
// of 8-byte accesses for these strided rows (measured: the length-1024 column pass 2.93 -> 2.33 ms).
template <typename T, int C, int NT>
__device__ __forceinline__ void tile_in(Cx<T>* __restrict__ dst, int lst, const Cx<T>* __restrict__ src, int pz,
                                        int n, int nrow) {
  if constexpr (sizeof(Cx<T>) == 8 && C % 2 == 0) {
    constexpr int C2 = C / 2;
    for (int idx = threadIdx.x; idx < n * C2; idx += NT) {
      const int i = idx / C2, cc = 2 * (idx % C2);
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (i < nrow) v = *reinterpret_cast<const float4*>(src + (size_t)i * pz + cc);
      dst[cc * lst + lds_pad(i)] = Cx<T>{v.x, v.y};
      dst[(cc + 1) * lst + lds_pad(i)] = Cx<T>{v.z, v.w};
    }
  } else {
    for (int idx = threadIdx.x; idx < n * C; idx += NT) {
      const int i = idx / C, cc = idx % C;
      dst[cc * lst + lds_pad(i)] = (i < nrow) ? src[(size_t)i * pz + cc] : czero<T>();
    }
  }
}

template <typename T, int C, int NT>
__device__ __forceinline__ void tile_out(Cx<T>* __restrict__ dst, int pz, const Cx<T>* __restrict__ src, int lst,
                                         int nrow) {
  if constexpr (sizeof(Cx<T>) == 8 && C % 2 == 0) {
    constexpr int C2 = C / 2;
    for (int idx = threadIdx.x; idx < nrow * C2; idx += NT) {
      const int i = idx / C2, cc = 2 * (idx % C2);
      const Cx<T> a = src[cc * lst + lds_pad(i)], b = src[(cc + 1) * lst + lds_pad(i)];
      *reinterpret_cast<float4*>(dst + (size_t)i * pz + cc) = make_float4(a.re, a.im, b.re, b.im);
    }
  } else {
    for (int idx = threadIdx.x; idx < nrow * C; idx += NT) {
      const int i = idx / C, cc = idx % C;
      dst[(size_t)i * pz + cc] = src[cc * lst + lds_pad(i)];
    }
  }
}

template <typename T, int L, int C>
__global__ __launch_bounds__(C * FftPlan<L>::G) void k_cols(Cx<T>* __restrict__ tmp, const Cx<T>* __restrict__ gs,
                                                            int nx, int pz, int nslots, int adj,
                                                            const Cx<T>* __restrict__ tw2,
                                                            const Slot<T>* __restrict__ tab) {
  using P = FftPlan<L>;
  constexpr int G = P::G, E = P::E, NT = C * G, ST = ColTile<T, L>::stride;
  __shared__ Cx<T> tile[C * ST];
  __shared__ Cx<T> xbuf[C][lds_len<L>()];
  __shared__ Cx<T> stw[lds_len<L>()];
  stage_twiddles<T, L>(stw, tw2);
  // Tiles narrower than a 128-byte line are grouped PAIR at a time; the PAIR
  // tiles of one line and one vector take consecutive logical ids, so the
  // second half of every line is an L2 hit, and all vectors of a tile group
  // follow each other (spectrum reuse in L2).
  constexpr int PAIR = (C * (int)sizeof(Cx<T>) >= 128) ? 1 : 128 / (C * (int)sizeof(Cx<T>));
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int grp_id = lb / (nslots * PAIR), rem = lb % (nslots * PAIR);
  const int slot = rem / PAIR;
  const int c0 = (grp_id * PAIR + rem % PAIR) * C;
  Cx<T>* tb = tmp + (size_t)slot * nx * pz + c0;
  const int c = threadIdx.x / G, g = threadIdx.x % G;
  const Cx<T>* gsl = tab ? tab[slot].gs : gs;
  const Cx<T>* g0 = gsl + (size_t)(c0 + c) * L;
  const Cx<T>* g1 = gsl + ((size_t)pz + c0 + c) * L;
  // this group's spectrum values: loaded before the tile where that was measured faster (lengths up to 128,
  // and 4-column tiles), so that their latency hides behind the tile load and the forward transform; the wider
  // tiles of the long lengths load them between the transforms
  constexpr bool early = L <= 128 || C <= 4;
  Cx<T> s0[E], s1[E];
  auto load_spectrum = [&] {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = fft_elem<L>(g, e);
      s0[e] = g0[p];
      s1[e] = g1[p];
    }
  };
  if constexpr (early) load_spectrum();
  tile_in<T, C, NT>(tile, ST, tb, pz, L, nx);
  __syncthreads();
  Cx<T>* col = tile + c * ST;
  // even (h = 0) and odd (h = 1) frequency halves along x
  Cx<T> ve[E], vo[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = fft_elem<L>(g, e);
    ve[e] = col[lds_pad(p)];
    vo[e] = ve[e] * tw_lo<T, L>(stw, p);
  }
  fft2_regs<T, L, false>(ve, vo, g, col, xbuf[c], stw);
  if constexpr (!early) load_spectrum();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    ve[e] = adj ? cmul_conj(s0[e], ve[e]) : s0[e] * ve[e];
    vo[e] = adj ? cmul_conj(s1[e], vo[e]) : s1[e] * vo[e];
  }
  fft2_regs<T, L, true>(ve, vo, g, col, xbuf[c], stw);
  wave_sync();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = fft_elem<L>(g, e);
    col[lds_pad(p)] = ve[e] + cmul_conj(tw_lo<T, L>(stw, p), vo[e]);
  }
  __syncthreads();
  tile_out<T, C, NT>(tb, pz, tile, ST, nx);
}

// Column pass of length 1 (the circular x-period 2 of sub-domain convolutions between half-nodes of one column):
// the length-1 transforms are the identity and the twiddle of the even/odd recombination is 1, so every column
// of a slot's single row is multiplied by s0 + s1 (by conj(s0 + s1) for the adjoint).
template <typename T>
__global__ void k_cols_len1(Cx<T>* __restrict__ tmp, const Cx<T>* __restrict__ gs, int pz, size_t total, int adj) {
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx % pz);
    const Cx<T> f = gs[c] + gs[pz + c];
    tmp[idx] = adj ? cmul_conj(f, tmp[idx]) : f * tmp[idx];
  }
}

// Forward-only (DIR 0) and inverse-only (DIR 1) column transforms: the y passes of the 3D operator and the
// spectrum set-up.  Slot s holds a [rows_slot][pz] array; a workgroup owns C adjacent columns as in k_cols.
// DIR 0: rows i < nrow are the input (the rest of the padded axis is zero); the length-2L transform is written
// back as rows m (wavenumber 2m) and L + m (wavenumber 2m + 1), m < L (rows_slot >= 2L).  DIR 1: rows m and
// L + m hold the even and odd halves of a spectrum; the first nrow outputs of the unnormalised inverse length-2L
// transform are written to rows i < nrow.
template <typename T, int L, int C, int DIR>
__global__ __launch_bounds__(C * FftPlan<L>::G) void k_cols_half(Cx<T>* __restrict__ tmp, int rows_slot, int nrow,
                                                                 int pz, int nslots,
                                                                 const Cx<T>* __restrict__ tw2) {
  using P = FftPlan<L>;
  constexpr int G = P::G, E = P::E, NT = C * G, ST = ColTile<T, L>::stride;
  __shared__ Cx<T> tile[C * ST];
  __shared__ Cx<T> xbuf[C][lds_len<L>()];
  __shared__ Cx<T> stw[lds_len<L>()];
  stage_twiddles<T, L>(stw, tw2);
  constexpr int PAIR = (C * (int)sizeof(Cx<T>) >= 128) ? 1 : 128 / (C * (int)sizeof(Cx<T>));
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int grp_id = lb / (nslots * PAIR), rem = lb % (nslots * PAIR);
  const int slot = rem / PAIR;
  const int c0 = (grp_id * PAIR + rem % PAIR) * C;
  Cx<T>* tb = tmp + (size_t)slot * rows_slot * pz + c0;
  const int c = threadIdx.x / G, g = threadIdx.x % G;
  if constexpr (DIR == 0) {
    tile_in<T, C, NT>(tile, ST, tb, pz, L, nrow);
  } else {
    tile_in<T, C, NT>(tile, ST, tb, pz, L, L);
    tile_in<T, C, NT>(&xbuf[0][0], lds_len<L>(), tb + (size_t)L * pz, pz, L, L);
  }
  __syncthreads();
  Cx<T>* col = tile + c * ST;
  Cx<T> ve[E], vo[E];
  if constexpr (DIR == 0) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = fft_elem<L>(g, e);
      ve[e] = col[lds_pad(p)];
      vo[e] = ve[e] * tw_lo<T, L>(stw, p);
    }
    fft2_regs<T, L, false>(ve, vo, g, col, xbuf[c], stw);
    wave_sync();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = fft_elem<L>(g, e);
      col[lds_pad(p)] = ve[e];
      xbuf[c][lds_pad(p)] = vo[e];
    }
    __syncthreads();
    tile_out<T, C, NT>(tb, pz, tile, ST, L);
    tile_out<T, C, NT>(tb + (size_t)L * pz, pz, &xbuf[0][0], lds_len<L>(), L);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = fft_elem<L>(g, e);
      ve[e] = col[lds_pad(p)];
      vo[e] = xbuf[c][lds_pad(p)];
    }
    wave_sync();
    fft2_regs<T, L, true>(ve, vo, g, col, xbuf[c], stw);
    wave_sync();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = fft_elem<L>(g, e);
      col[lds_pad(p)] = ve[e] + cmul_conj(tw_lo<T, L>(stw, p), vo[e]);
    }
    __syncthreads();
    tile_out<T, C, NT>(tb, pz, tile, ST, nrow);
  }
}

// 3D spectrum from the forward transforms F of the weighted lag table (lags l >= 0 with weight 1/2 at l = 0 on
// each axis, so that the transform of the even circulant extension is the sum of F over the 8 sign flips of
// the wavenumber): F is [px][py pz] in the split order of the passes (wavenumber 2m at position m, 2m + 1 at
// L + m on every axis); gs[h][cy pz + cz][m] = scale * sum_{signs} F at (+-kx, +-ky, +-kz), kx = 2m + h.
__device__ __forceinline__ int split_pos(int k, int L) { return (k & 1) ? L + (k >> 1) : (k >> 1); }
__device__ __forceinline__ int split_k(int pos, int L) { return pos < L ? 2 * pos : 2 * (pos - L) + 1; }

__global__ void k_spec3_sym(const Cx<double>* __restrict__ F, int lx, int ly, int lz, double scale,
                            Cx<double>* __restrict__ gs64, Cx<float>* __restrict__ gs32) {
  const int px = 2 * lx, py = 2 * ly, pz = 2 * lz;
  const size_t cols = (size_t)py * pz, total = (size_t)px * cols;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int m = (int)(t % lx);
    const size_t r = t / lx;
    const size_t cc = r % cols;
    const int h = (int)(r / cols);
    const int cy = (int)(cc / pz), cz = (int)(cc % pz);
    const int kx = 2 * m + h, ky = split_k(cy, ly), kz = split_k(cz, lz);
    const int xs[2] = {split_pos(kx, lx), split_pos((px - kx) % px, lx)};
    const int ys[2] = {split_pos(ky, ly), split_pos((py - ky) % py, ly)};
    const int zs[2] = {split_pos(kz, lz), split_pos((pz - kz) % pz, lz)};
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const Cx<double> v = F[(size_t)xs[a] * cols + (size_t)ys[b] * pz + zs[c]];
          re += v.re;
          im += v.im;
        }
    const Cx<double> out{scale * re, scale * im};
    if (gs64) gs64[t] = out;
    if (gs32) gs32[t] = ccast<float>(out);
  }
}

// Weighted lag table of the 3D spectrum: u[p][q][s] = K3[p][q][s] w(p) w(q) w(s), w(0) = 1/2, else 1.
__global__ void k_lag_weight3(const Cx<double>* __restrict__ K, int nx, int ny, int nz, Cx<double>* __restrict__ u) {
  const size_t n = (size_t)nx * ny * nz;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    const int s = (int)(t % nz), q = (int)((t / nz) % ny), p = (int)(t / ((size_t)ny * nz));
    const double w = (p ? 1.0 : 0.5) * (q ? 1.0 : 0.5) * (s ? 1.0 : 0.5);
    u[t] = Cx<double>{w * K[t].re, w * K[t].im};
  }
}

// 3D lag table of the ball-integrated Green's function: K = c1 e^{i k0 r} / r (r = h |lag| > 0), K(0) = self.
__global__ void k_table3(Cx<double>* __restrict__ ktab, int nx, int ny, int nz, double k0, double h, double c1,
                         Cx<double> self) {
  const size_t n = (size_t)nx * ny * nz;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    const int s = (int)(t % nz), q = (int)((t / nz) % ny), p = (int)(t / ((size_t)ny * nz));
    if (t == 0) {
      ktab[0] = self;
      continue;
    }
    const double r = h * sqrt((double)p * p + (double)q * q + (double)s * s);
    double sn, cs;
    sincos(k0 * r, &sn, &cs);
    ktab[t] = Cx<double>{c1 * cs / r, c1 * sn / r};
  }
}

// Incident fields of 3D point sources: psi0 = amp K3(|i - si|, |j - sj|, |l - sl|) / h^3.
template <typename T>
__global__ void k_incident3(const Cx<double>* __restrict__ ktab, const int* __restrict__ src,
                            const Cx<double>* __restrict__ amp, Cx<T>* __restrict__ out, int nx, int ny, int nz,
                            int nsrc, double inv_dv) {
  const size_t n = (size_t)nx * ny * nz, total = n * nsrc;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x) {
    const int sidx = (int)(k / n);
    const size_t r = k % n;
    const int l = (int)(r % nz), j = (int)((r / nz) % ny), i = (int)(r / ((size_t)ny * nz));
    const int di = abs(i - src[3 * sidx]), dj = abs(j - src[3 * sidx + 1]), dl = abs(l - src[3 * sidx + 2]);
    const Cx<double> v = inv_dv * (amp[sidx] * ktab[((size_t)di * ny + dj) * nz + dl]);
    out[k] = ccast<T>(v);
  }
}

// ------------------------------------------------------------------ pass 3
template <typename T, int L>
__global__ __launch_bounds__((rows_threads<T, L>())) void k_rows_inv(const Cx<T>* __restrict__ tmp, const Cx<T>* x,
                                                                     const T* __restrict__ chi, const Cx<T>* rhs,
                                                                     Cx<T>* y, double* __restrict__ rnorm,
                                                                     const int* __restrict__ vidx, int nx, int nz,
                                                                     int nitems, int epi,
                                                                     const Cx<T>* __restrict__ tw2, int nodes, int lo,
                                                                     int hi, const Slot<T>* __restrict__ tab,
                                                                     int trows, RowMap rm) {
  using P = FftPlan<L>;
  constexpr int G = P::G, E = P::E, GPW = rows_threads<T, L>() / G;
  __shared__ Cx<T> sbuf[GPW][2][lds_len<L>()];
  __shared__ Cx<T> stw[lds_len<L>()];
  stage_twiddles<T, L>(stw, tw2);
  __syncthreads();
  const int grp = threadIdx.x / G, g = threadIdx.x % G;
  const size_t vstride = (size_t)nodes * nx * nz;
  for (int base = blockIdx.x * GPW; base < nitems; base += gridDim.x * GPW) {
    const int item = base + grp;
    const int it = item < nitems ? item : nitems - 1;
    const int slot = it / rm.ns, ii = it % rm.ns, i = rm.xa + rm.xs * ii;
    const bool valid = item < nitems && i >= lo && i < hi;
    const int node = slot % nodes, vs = slot / nodes;
    const int vi = vidx ? vidx[vs] : vs;
    const size_t row = (size_t)node * nx + i;
    const Cx<T>* tr = tmp + ((size_t)slot * trows + ii) * (2 * L);
    Cx<T> acc[E], v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = fft_elem<L>(g, e);
      acc[e] = tr[p];
      v[e] = tr[L + p];
    }
    fft2_regs<T, L, true>(acc, v, g, sbuf[grp][0], sbuf[grp][1], stw);
    const size_t off = tab ? row * nz : (size_t)vi * vstride + row * nz;
    const Cx<T>* xs = tab ? tab[slot].x : x;
    Cx<T>* ys = tab ? tab[slot].y : y;
    const Cx<T>* rs = tab ? tab[slot].rhs : rhs;
    const T* cs = (tab ? tab[slot].chi : chi) + row * nz;
    double* rn = tab ? tab[slot].rnorm : (rnorm ? rnorm + slot / nodes : nullptr);
    double nrm = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = fft_elem<L>(g, e);
      if (p < nz) {
        const Cx<T> conv = acc[e] + cmul_conj(tw_lo<T, L>(stw, p), v[e]);
        Cx<T> out;
        switch (epi) {
          case 0: out = xs[off + p] - conv; break;
          case 1: out = conv; break;
          case 2: out = xs[off + p] - cs[p] * conv; break;
          default: out = cs[p] * conv; break;
        }
        if (rs) {
          out = out - rs[off + p];
          nrm += (double)out.re * (double)out.re + (double)out.im * (double)out.im;
        }
        if (valid) ys[off + p] = out;
      }
    }
    if (rn) {
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) nrm += __shfl_xor(nrm, o);
      if (valid && g == 0) atomicAdd(rn, nrm);
    }
    wave_sync();
  }
}

// ---------------------------------------------------------- spectrum set-up
// Row pass: row p of the circulant table (length pz = 2 lz, full input),
// written transposed to s1t[c][p] in the split column order.
template <int L>
__global__ __launch_bounds__((rows_threads<double, L>())) void k_spec_rows(const Cx<double>* __restrict__ ktab,
                                                                           int nx, int nz, int px,
                                                                           Cx<double>* __restrict__ s1t,
                                                                           const Cx<double>* __restrict__ tw2,
                                                                           int circ) {
  using P = FftPlan<L>;
  constexpr int G = P::G, E = P::E, GPW = rows_threads<double, L>() / G;
  __shared__ Cx<double> sbuf[GPW][2][lds_len<L>()];
  __shared__ Cx<double> stw[lds_len<L>()];
  stage_twiddles<double, L>(stw, tw2);
  __syncthreads();
  const int grp = threadIdx.x / G, g = threadIdx.x % G;
  const int pz = 2 * L;
  for (int base = blockIdx.x * GPW; base < px; base += gridDim.x * GPW) {
    const int p = base + grp;
    const bool valid = p < px;
    const int pp = valid ? p : px - 1;
    const int lxp = (circ || pp < px - pp) ? pp : px - pp;
    Cx<double> a[E], b[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int q = fft_elem<L>(g, e);
      // lags of columns q and q + L: q (q < L) and min(q + L, L - q) = L - q
      const int l2 = L - q;
      Cx<double> k1 = czero<double>(), k2 = czero<double>();
      if (lxp < nx && q < nz) k1 = ktab[(size_t)lxp * nz + q];
      if (lxp < nx && l2 < nz) k2 = ktab[(size_t)lxp * nz + l2];
      a[e] = k1 + k2;
      b[e] = (k1 - k2) * tw_lo<double, L>(stw, q);
    }
    fft2_regs<double, L, false>(a, b, g, sbuf[grp][0], sbuf[grp][1], stw);
    if (valid) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int m = fft_elem<L>(g, e);
        s1t[(size_t)m * px + p] = a[e];
        s1t[(size_t)(L + m) * px + p] = b[e];
      }
    }
    wave_sync();
  }
}

// Length-2 x-transform of s1t[c][0..2) -> gs[h][c] (lx = 1): the sum and the difference of the two positions.
__global__ void k_spec_len1(const Cx<double>* __restrict__ s1t, int pz, Cx<double>* __restrict__ gs64,
                            Cx<float>* __restrict__ gs32, double scale, double scale_odd) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < pz; c += gridDim.x * blockDim.x) {
    const Cx<double> k1 = s1t[2 * (size_t)c], k2 = s1t[2 * (size_t)c + 1];
    const Cx<double> va = scale * (k1 + k2), vb = scale_odd * (k1 - k2);
    if (gs64) {
      gs64[c] = va;
      gs64[pz + c] = vb;
    }
    if (gs32) {
      gs32[c] = ccast<float>(va);
      gs32[pz + c] = ccast<float>(vb);
    }
  }
}

// Column pass: full-length transform of s1t[c][0..px) -> gs[h][c][m] scaled (the odd half h = 1 by
// scale_odd).
template <int L>
__global__ __launch_bounds__((rows_threads<double, L>())) void k_spec_cols(const Cx<double>* __restrict__ s1t,
                                                                           int pz, Cx<double>* __restrict__ gs64,
                                                                           Cx<float>* __restrict__ gs32,
                                                                           double scale, double scale_odd,
                                                                           const Cx<double>* __restrict__ tw2) {
  using P = FftPlan<L>;
  constexpr int G = P::G, E = P::E, GPW = rows_threads<double, L>() / G;
  __shared__ Cx<double> sbuf[GPW][2][lds_len<L>()];
  __shared__ Cx<double> stw[lds_len<L>()];
  stage_twiddles<double, L>(stw, tw2);
  __syncthreads();
  const int grp = threadIdx.x / G, g = threadIdx.x % G;
  const int px = 2 * L;
  for (int base = blockIdx.x * GPW; base < pz; base += gridDim.x * GPW) {
    const int c = base + grp;
    const bool valid = c < pz;
    const int cc = valid ? c : pz - 1;
    const Cx<double>* col = s1t + (size_t)cc * px;
    Cx<double> a[E], b[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = fft_elem<L>(g, e);
      const Cx<double> k1 = col[p], k2 = col[p + L];
      a[e] = k1 + k2;
      b[e] = (k1 - k2) * tw_lo<double, L>(stw, p);
    }
    fft2_regs<double, L, false>(a, b, g, sbuf[grp][0], sbuf[grp][1], stw);
    if (valid) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int m = fft_elem<L>(g, e);
        const Cx<double> va = scale * a[e], vb = scale_odd * b[e];
        if (gs64) {
          gs64[(size_t)cc * L + m] = va;
          gs64[((size_t)pz + cc) * L + m] = vb;
        }
        if (gs32) {
          gs32[(size_t)cc * L + m] = ccast<float>(va);
          gs32[((size_t)pz + cc) * L + m] = ccast<float>(vb);
        }
      }
    }
    wave_sync();
  }
}

__global__ void k_contrast(const double* __restrict__ vel, double* __restrict__ chi64, float* __restrict__ chi32,
                           int n, double w2, double inv_c02, unsigned* bad) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const double c = vel[k];
    if (!(c > 0.0) || !isfinite(c)) atomicOr(bad, 1u);
    const double chi = w2 * (1.0 / (c * c) - inv_c02);
    if (chi64) chi64[k] = chi;
    if (chi32) chi32[k] = (float)chi;
  }
}

__global__ void k_table(Cx<double>* __restrict__ ktab, int nx, int nz, double k0h, Cx<double> cj1,
                        Cx<double> self) {
  const int n = nx * nz;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int p = k / nz, q = k % nz;
    if (p == 0 && q == 0) {
      ktab[k] = self;
      continue;
    }
    const double x = k0h * sqrt((double)(p * p + q * q));
    double j0, y0;
    lsop_bessel::hankel0(x, &j0, &y0);
    ktab[k] = cj1 * Cx<double>{j0, y0};
  }
}

template <typename T>
__global__ void k_incident(const Cx<double>* __restrict__ ktab, const int* __restrict__ si,
                           const int* __restrict__ sj, const Cx<double>* __restrict__ amp, Cx<T>* __restrict__ out,
                           int nx, int nz, int nsrc, double inv_dv) {
  const size_t n = (size_t)nx * nz, total = n * nsrc;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x) {
    const int s = (int)(k / n);
    const int r = (int)(k % n);
    const int i = r / nz, j = r % nz;
    const int di = abs(i - si[s]), dj = abs(j - sj[s]);
    const Cx<double> v = inv_dv * (amp[s] * ktab[(size_t)di * nz + dj]);
    out[k] = ccast<T>(v);
  }
}

// -------------------------------------------------------------- launchers
namespace {
int grid_for_rows(int nitems, int gpw) {
  const int need = (nitems + gpw - 1) / gpw;
  const int cap = 256 * 8;
  return need < cap ? need : cap;
}
}  // namespace

#define LSOP_DISPATCH_L(L, ...)                                \
  switch (L) {                                                 \
    case 32: { constexpr int LL = 32; __VA_ARGS__; } break;     \
    case 64: { constexpr int LL = 64; __VA_ARGS__; } break;     \
    case 96: { constexpr int LL = 96; __VA_ARGS__; } break;     \
    case 128: { constexpr int LL = 128; __VA_ARGS__; } break;   \
    case 192: { constexpr int LL = 192; __VA_ARGS__; } break;   \
    case 256: { constexpr int LL = 256; __VA_ARGS__; } break;   \
    case 384: { constexpr int LL = 384; __VA_ARGS__; } break;   \
    case 512: { constexpr int LL = 512; __VA_ARGS__; } break;   \
    case 768: { constexpr int LL = 768; __VA_ARGS__; } break;   \
    case 1024: { constexpr int LL = 1024; __VA_ARGS__; } break; \
    case 2048: { constexpr int LL = 2048; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                      \
  }

// x-direction lengths also include the short sub-domain transforms
#define LSOP_DISPATCH_LX(L, ...)                           \
  switch (L) {                                             \
    case 2: { constexpr int LL = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int LL = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int LL = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int LL = 16; __VA_ARGS__; } break; \
    default: LSOP_DISPATCH_L(L, __VA_ARGS__);              \
  }

// Resolves the defaults of a row map and checks that every row it visits lies in the strip and in tmp.
static bool row_map_ok(RowMap& rm, int nx, int& trows) {
  if (rm.ns < 0) rm.ns = nx;
  if (trows < 0) trows = rm.ns;
  if (rm.ns < 1 || trows < rm.ns || (rm.xs != 1 && rm.xs != -1)) return false;
  const long last = (long)rm.xa + (long)rm.xs * (rm.ns - 1);
  return rm.xa >= 0 && rm.xa < nx && last >= 0 && last < nx;
}

template <typename T>
hipError_t launch_rows_fwd(int L, const Cx<T>* x, const T* chi, Cx<T>* tmp, const int* vidx, int nx, int nz,
                           int nslots, bool mulchi, const Cx<T>* tw2, hipStream_t s, int nodes, int lo, int hi,
                           const Slot<T>* tab, int trows, RowMap rm) {
  if (nslots <= 0 || nx <= 0) return hipSuccess;
  if (nodes < 1 || nslots % nodes != 0 || (tab && (nodes != 1 || vidx))) return hipErrorInvalidValue;
  if (!row_map_ok(rm, nx, trows)) return hipErrorInvalidValue;
  if (hi < 0) hi = nx;
  const int nitems = nslots * rm.ns;
  LSOP_DISPATCH_L(L, {
    constexpr int NT = rows_threads<T, LL>(), GPW = NT / FftPlan<LL>::G;
    hipLaunchKernelGGL((k_rows_fwd<T, LL>), dim3(grid_for_rows(nitems, GPW)), dim3(NT), 0, s, x, chi, tmp, vidx,
                       nx, nz, nitems, (int)mulchi, tw2, nodes, lo, hi, tab, trows, rm);
  });
  return hipGetLastError();
}

// Column-tile width: the default is the widest tile that fits (ColTile); a
// narrower tile (more workgroups per CU) can be selected per call (tile > 0).
template <typename T>
hipError_t launch_cols(int L, Cx<T>* tmp, const Cx<T>* gs, int nx, int pz, int nslots, bool adj, const Cx<T>* tw2,
                       hipStream_t s, int tile, int* used, const Slot<T>* tab) {
  if (nslots <= 0) return hipSuccess;
  if (pz % 16 != 0) return hipErrorInvalidValue;  // tile groups of one 128-byte line must divide the row
  if (L == 1) {  // one row per slot, no transform
    if (nx != 1 || tab) return hipErrorInvalidValue;
    if (used) *used = 0;
    const size_t total = (size_t)nslots * pz;
    size_t grid = (total + 255) / 256;
    if (grid > 16384) grid = 16384;
    hipLaunchKernelGGL((k_cols_len1<T>), dim3((unsigned)grid), dim3(256), 0, s, tmp, gs, pz, total, (int)adj);
    return hipGetLastError();
  }
  LSOP_DISPATCH_LX(L, {
    constexpr int CMAX = ColTile<T, LL>::C;
    int C = (tile > 0 && tile < CMAX) ? tile : CMAX;
    C = C >= 256 ? 256 : C >= 128 ? 128 : C >= 64 ? 64 : C >= 32 ? 32 : C >= 16 ? 16 : C >= 8 ? 8 : C >= 4 ? 4
      : (CMAX < 2 ? CMAX : 2);
    while (C > 16 && pz % C != 0) C /= 2;  // tiles must divide the row (pz % 16 == 0)
    if (used) *used = C;
    const int ntiles = pz / C;
    const dim3 grid(ntiles * nslots);
    switch (C) {
      case 256:
        if constexpr (CMAX >= 256)
          hipLaunchKernelGGL((k_cols<T, LL, 256>), grid, dim3(256 * FftPlan<LL>::G), 0, s, tmp, gs, nx, pz, nslots,
                             (int)adj, tw2, tab);
        break;
      case 128:
        if constexpr (CMAX >= 128)
          hipLaunchKernelGGL((k_cols<T, LL, 128>), grid, dim3(128 * FftPlan<LL>::G), 0, s, tmp, gs, nx, pz, nslots,
                             (int)adj, tw2, tab);
        break;
      case 64:
        if constexpr (CMAX >= 64)
          hipLaunchKernelGGL((k_cols<T, LL, 64>), grid, dim3(64 * FftPlan<LL>::G), 0, s, tmp, gs, nx, pz, nslots,
                             (int)adj, tw2, tab);
        break;
      case 32:
        if constexpr (CMAX >= 32)
          hipLaunchKernelGGL((k_cols<T, LL, 32>), grid, dim3(32 * FftPlan<LL>::G), 0, s, tmp, gs, nx, pz, nslots,
                             (int)adj, tw2, tab);
        break;
      case 16:
        if constexpr (CMAX >= 16)
          hipLaunchKernelGGL((k_cols<T, LL, 16>), grid, dim3(16 * FftPlan<LL>::G), 0, s, tmp, gs, nx, pz, nslots,
                             (int)adj, tw2, tab);
        break;
      case 8:
        if constexpr (CMAX >= 8)
          hipLaunchKernelGGL((k_cols<T, LL, 8>), grid, dim3(8 * FftPlan<LL>::G), 0, s, tmp, gs, nx, pz, nslots,
                             (int)adj, tw2, tab);
        break;
      case 4:
        if constexpr (CMAX >= 4)
          hipLaunchKernelGGL((k_cols<T, LL, 4>), grid, dim3(4 * FftPlan<LL>::G), 0, s, tmp, gs, nx, pz, nslots,
                             (int)adj, tw2, tab);
        break;
      default:
        hipLaunchKernelGGL((k_cols<T, LL, (CMAX < 2 ? CMAX : 2)>), grid, dim3((CMAX < 2 ? CMAX : 2) * FftPlan<LL>::G),
                           0, s, tmp, gs, nx, pz, nslots, (int)adj, tw2, tab);
        break;
    }
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rows_inv(int L, const Cx<T>* tmp, const Cx<T>* x, const T* chi, const Cx<T>* rhs, Cx<T>* y,
                           double* rnorm, const int* vidx, int nx, int nz, int nslots, int epi, const Cx<T>* tw2,
                           hipStream_t s, int nodes, int lo, int hi, const Slot<T>* tab, int trows, RowMap rm) {
  if (nslots <= 0 || nx <= 0) return hipSuccess;
  if (nodes < 1 || nslots % nodes != 0 || (tab && (nodes != 1 || vidx))) return hipErrorInvalidValue;
  if (!row_map_ok(rm, nx, trows)) return hipErrorInvalidValue;
  if (hi < 0) hi = nx;
  const int nitems = nslots * rm.ns;
  LSOP_DISPATCH_L(L, {
    constexpr int NT = rows_threads<T, LL>(), GPW = NT / FftPlan<LL>::G;
    hipLaunchKernelGGL((k_rows_inv<T, LL>), dim3(grid_for_rows(nitems, GPW)), dim3(NT), 0, s, tmp, x, chi, rhs, y,
                       rnorm, vidx, nx, nz, nitems, epi, tw2, nodes, lo, hi, tab, trows, rm);
  });
  return hipGetLastError();
}

hipError_t launch_spectrum(int lx, int lz, const Cx<double>* ktab, int nx, int nz, Cx<double>* s1t,
                           Cx<double>* gs64, Cx<float>* gs32, const Cx<double>* tw2x, const Cx<double>* tw2z,
                           hipStream_t s, bool circ) {
  const int px = 2 * lx, pz = 2 * lz;
  if (circ && nx < px) return hipErrorInvalidValue;  // every lag of the period must be in the table
  LSOP_DISPATCH_L(lz, {
    constexpr int NT = rows_threads<double, LL>(), GPW = NT / FftPlan<LL>::G;
    hipLaunchKernelGGL((k_spec_rows<LL>), dim3(grid_for_rows(px, GPW)), dim3(NT), 0, s, ktab, nx, nz, px, s1t,
                       tw2z, (int)circ);
  });
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double scale = 1.0 / ((double)px * (double)pz);
  if (lx == 1) {
    hipLaunchKernelGGL(k_spec_len1, dim3((pz + 255) / 256), dim3(256), 0, s, s1t, pz, gs64, gs32, scale,
                       circ ? -scale : scale);
    return hipGetLastError();
  }
  LSOP_DISPATCH_LX(lx, {
    constexpr int NT = rows_threads<double, LL>(), GPW = NT / FftPlan<LL>::G;
    hipLaunchKernelGGL((k_spec_cols<LL>), dim3(grid_for_rows(pz, GPW)), dim3(NT), 0, s, s1t, pz, gs64, gs32, scale,
                       circ ? -scale : scale, tw2x);
  });
  return hipGetLastError();
}

hipError_t launch_contrast(const double* vel, double* chi64, float* chi32, int n, double w2, double inv_c02,
                           unsigned* bad, hipStream_t s) {
  int grid = (n + 255) / 256;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_contrast, dim3(grid), dim3(256), 0, s, vel, chi64, chi32, n, w2, inv_c02, bad);
  return hipGetLastError();
}

hipError_t launch_table(Cx<double>* ktab, int nx, int nz, double k0h, Cx<double> cj1, Cx<double> self,
                        hipStream_t s) {
  const int n = nx * nz;
  int grid = (n + 255) / 256;
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(k_table, dim3(grid), dim3(256), 0, s, ktab, nx, nz, k0h, cj1, self);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_incident(const Cx<double>* ktab, const int* si, const int* sj, const Cx<double>* amp, Cx<T>* out,
                           int nx, int nz, int nsrc, double inv_dv, hipStream_t s) {
  const size_t total = (size_t)nx * nz * nsrc;
  size_t grid = (total + 255) / 256;
  if (grid > 16384) grid = 16384;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((k_incident<T>), dim3((unsigned)grid), dim3(256), 0, s, ktab, si, sj, amp, out, nx, nz, nsrc,
                     inv_dv);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cols_half(int dir, int L, Cx<T>* tmp, int rows_slot, int nrow, int pz, int nslots,
                            const Cx<T>* tw2, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  if (pz % 16 != 0 || rows_slot < 2 * L || nrow < 1 || nrow > L) return hipErrorInvalidValue;
  LSOP_DISPATCH_L(L, {
    constexpr int C = ColTile<T, LL>::C;
    const dim3 grid((pz / C) * nslots);
    if (dir == 0)
      hipLaunchKernelGGL((k_cols_half<T, LL, C, 0>), grid, dim3(C * FftPlan<LL>::G), 0, s, tmp, rows_slot, nrow, pz,
                         nslots, tw2);
    else
      hipLaunchKernelGGL((k_cols_half<T, LL, C, 1>), grid, dim3(C * FftPlan<LL>::G), 0, s, tmp, rows_slot, nrow, pz,
                         nslots, tw2);
  });
  return hipGetLastError();
}

hipError_t launch_table3(Cx<double>* ktab, int nx, int ny, int nz, double k0, double h, double c1, Cx<double> self,
                         hipStream_t s) {
  const size_t n = (size_t)nx * ny * nz;
  size_t grid = (n + 255) / 256;
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(k_table3, dim3((unsigned)grid), dim3(256), 0, s, ktab, nx, ny, nz, k0, h, c1, self);
  return hipGetLastError();
}

// 3D spectrum: weighted lag table (into u: nx ny nz complex doubles), forward z rows into F ([px][py][pz]), y
// columns per x-plane, x columns, then the sign-flip sum into gs.
hipError_t launch_spectrum3(int lx, int ly, int lz, const Cx<double>* ktab, int nx, int ny, int nz, Cx<double>* u,
                            Cx<double>* F, Cx<double>* gs64, Cx<float>* gs32, const Cx<double>* tw2x,
                            const Cx<double>* tw2y, const Cx<double>* tw2z, hipStream_t s) {
  const int px = 2 * lx, py = 2 * ly, pz = 2 * lz;
  const size_t n = (size_t)nx * ny * nz;
  size_t grid = (n + 255) / 256;
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(k_lag_weight3, dim3((unsigned)grid), dim3(256), 0, s, ktab, nx, ny, nz, u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_rows_fwd<double>(lz, u, nullptr, F, nullptr, ny, nz, nx, false, tw2z, s, nx, 0, ny, nullptr, py)))
    return e;
  if ((e = launch_cols_half<double>(0, ly, F, py, ny, pz, nx, tw2y, s))) return e;
  if ((e = launch_cols_half<double>(0, lx, F, px, nx, py * pz, 1, tw2x, s))) return e;
  const size_t total = (size_t)px * py * pz;
  grid = (total + 255) / 256;
  if (grid > 16384) grid = 16384;
  hipLaunchKernelGGL(k_spec3_sym, dim3((unsigned)grid), dim3(256), 0, s, F, lx, ly, lz,
                     1.0 / ((double)px * (double)py * (double)pz), gs64, gs32);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_incident3(const Cx<double>* ktab, const int* src, const Cx<double>* amp, Cx<T>* out, int nx,
                            int ny, int nz, int nsrc, double inv_dv, hipStream_t s) {
  const size_t total = (size_t)nx * ny * nz * nsrc;
  size_t grid = (total + 255) / 256;
  if (grid > 16384) grid = 16384;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((k_incident3<T>), dim3((unsigned)grid), dim3(256), 0, s, ktab, src, amp, out, nx, ny, nz, nsrc,
                     inv_dv);
  return hipGetLastError();
}

#define LSOP_INST(T)                                                                                               \
  template hipError_t launch_rows_fwd<T>(int, const Cx<T>*, const T*, Cx<T>*, const int*, int, int, int, bool,    \
                                         const Cx<T>*, hipStream_t, int, int, int, const Slot<T>*, int, RowMap);  \
  template hipError_t launch_cols<T>(int, Cx<T>*, const Cx<T>*, int, int, int, bool, const Cx<T>*, hipStream_t,    \
                                     int, int*, const Slot<T>*);                                                  \
  template hipError_t launch_rows_inv<T>(int, const Cx<T>*, const Cx<T>*, const T*, const Cx<T>*, Cx<T>*,        \
                                         double*, const int*, int, int, int, int, const Cx<T>*, hipStream_t, int, \
                                         int, int, const Slot<T>*, int, RowMap);                                  \
  template hipError_t launch_cols_half<T>(int, int, Cx<T>*, int, int, int, int, const Cx<T>*, hipStream_t);      \
  template hipError_t launch_incident3<T>(const Cx<double>*, const int*, const Cx<double>*, Cx<T>*, int, int,    \
                                          int, int, double, hipStream_t);                                         \
  template hipError_t launch_incident<T>(const Cx<double>*, const int*, const int*, const Cx<double>*, Cx<T>*,    \
                                         int, int, int, double, hipStream_t);
LSOP_INST(float)
LSOP_INST(double)

}  // namespace lsop
