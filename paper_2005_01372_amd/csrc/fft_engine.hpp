// Register/LDS Stockham FFT engine for gfx950.
//
// One FFT of length L is computed by a group of G lanes of a single wavefront
// (G <= 64), so the exchanges between radix stages only need wavefront-level
// ordering, never a workgroup barrier.  Each lane keeps E = L / G values in
// registers.  A stage with radix R and span Ns (product of the earlier radices)
// lets every lane run E / R radix-R butterflies b = g + G*u: the inputs of
// butterfly b are the elements b + r*(L/R) (r < R); they are twiddled by
// w_{Ns R}^{r (b mod Ns)}, transformed by a length-R DFT in registers, and
// written to positions (b / Ns) Ns R + (b mod Ns) + r Ns (the self-sorting
// Stockham formulation, Govindaraju et al., SC 2008).  The output is in
// natural order.
//
// Every plan starts and ends with the same radix, so the register <-> element
// map of the first stage's inputs equals that of the last stage's outputs:
//   element(e) = g + G*(e / R1) + (e % R1) * (L / R1),   e < E.
// A forward FFT, a pointwise multiply and an inverse FFT therefore chain in
// registers with no reordering, and both global loads and stores through this
// map are coalesced across lanes.
#pragma once
#include "cx.hpp"

template <int L>
struct FftPlan;
#define LSOP_FFT_PLAN(Lv, Gv, ...)                                   \
  template <>                                                        \
  struct FftPlan<Lv> {                                               \
    static constexpr int G = Gv;                                     \
    static constexpr int R[] = {__VA_ARGS__};                        \
    static constexpr int NST = sizeof(R) / sizeof(int);              \
    static constexpr int E = Lv / Gv;                                \
  };
// short lengths: the x-transforms of narrow sub-domains (hierarchical build)
LSOP_FFT_PLAN(2, 1, 2)
LSOP_FFT_PLAN(4, 1, 4)
LSOP_FFT_PLAN(8, 1, 8)
LSOP_FFT_PLAN(16, 4, 4, 4)
LSOP_FFT_PLAN(32, 8, 4, 2, 4)
LSOP_FFT_PLAN(64, 8, 8, 8)
LSOP_FFT_PLAN(96, 8, 4, 3, 2, 4)
LSOP_FFT_PLAN(128, 16, 4, 8, 4)
LSOP_FFT_PLAN(192, 8, 8, 3, 8)
LSOP_FFT_PLAN(256, 32, 8, 4, 8)
LSOP_FFT_PLAN(384, 16, 4, 3, 8, 4)
LSOP_FFT_PLAN(512, 64, 8, 8, 8)
LSOP_FFT_PLAN(768, 32, 8, 3, 4, 8)
LSOP_FFT_PLAN(1024, 64, 8, 16, 8)
LSOP_FFT_PLAN(2048, 64, 16, 8, 16)
#undef LSOP_FFT_PLAN

// LDS slot index with one element of padding every 16 (spreads strided
// Stockham stores over the banks).
__host__ __device__ constexpr int lds_pad(int p) { return p + (p >> 4); }
template <int L>
__host__ __device__ constexpr int lds_len() { return L + L / 16; }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- small DFTs
// Forward DFTs use w_R = exp(-2 pi i / R); INV uses the conjugate root.
template <typename T, bool INV>
__device__ __forceinline__ void dft2(Cx<T>* a) {
  Cx<T> t = a[0];
  a[0] = t + a[1];
  a[1] = t - a[1];
}

template <typename T, bool INV>
__device__ __forceinline__ void dft3(Cx<T>* a) {
  const T c = T(-0.5), s = T(0.866025403784438646763723170752936183);
  Cx<T> t = a[1] + a[2];
  Cx<T> d = a[1] - a[2];
  Cx<T> m = a[0] + c * t;
  // w3 = c - i s (forward): y1 = m - i s d, y2 = m + i s d
  Cx<T> sd = mul_mi<T, INV>(s * d);
  a[0] = a[0] + t;
  a[1] = m + sd;
  a[2] = m - sd;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(Cx<T>* a) {
  Cx<T> t0 = a[0] + a[2], t1 = a[0] - a[2];
  Cx<T> t2 = a[1] + a[3], t3 = mul_mi<T, INV>(a[1] - a[3]);
  a[0] = t0 + t2;
  a[2] = t0 - t2;
  a[1] = t1 + t3;
  a[3] = t1 - t3;
}

// multiply by w_8^k (forward sign) or its conjugate
template <typename T, bool INV, int K>
__device__ __forceinline__ Cx<T> w8(Cx<T> x) {
  const T h = T(0.707106781186547524400844362104849039);
  if constexpr (K == 0) return x;
  else if constexpr (K == 1) {
    // (1 - i)/sqrt2 forward, (1 + i)/sqrt2 inverse
    if constexpr (INV) return {h * (x.re - x.im), h * (x.re + x.im)};
    else return {h * (x.re + x.im), h * (x.im - x.re)};
  } else if constexpr (K == 2) return mul_mi<T, INV>(x);
  else {
    // (-1 - i)/sqrt2 forward, (-1 + i)/sqrt2 inverse
    if constexpr (INV) return {-h * (x.re + x.im), h * (x.re - x.im)};
    else return {h * (x.im - x.re), -h * (x.re + x.im)};
  }
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(Cx<T>* a) {
  Cx<T> e[4] = {a[0], a[2], a[4], a[6]};
  Cx<T> o[4] = {a[1], a[3], a[5], a[7]};
  dft4<T, INV>(e);
  dft4<T, INV>(o);
  o[1] = w8<T, INV, 1>(o[1]);
  o[2] = w8<T, INV, 2>(o[2]);
  o[3] = w8<T, INV, 3>(o[3]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a[k] = e[k] + o[k];
    a[k + 4] = e[k] - o[k];
  }
}

template <typename T, bool INV>
__device__ __forceinline__ void dft16(Cx<T>* a) {
  Cx<T> e[8], o[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    e[k] = a[2 * k];
    o[k] = a[2 * k + 1];
  }
  dft8<T, INV>(e);
  dft8<T, INV>(o);
  // w16^k = cos(k pi/8) -+ i sin(k pi/8)
  const T c1 = T(0.923879532511286756128183189396788933);
  const T s1 = T(0.382683432365089771728459984030398866);
  const T sg = INV ? T(1) : T(-1);
  const Cx<T> w[8] = {{T(1), T(0)}, {c1, sg * s1}, {T(0.707106781186547524400844362104849039), sg * T(0.707106781186547524400844362104849039)},
                      {s1, sg * c1}, {T(0), sg}, {-s1, sg * c1},
                      {T(-0.707106781186547524400844362104849039), sg * T(0.707106781186547524400844362104849039)}, {-c1, sg * s1}};
#pragma unroll
  for (int k = 1; k < 8; ++k) o[k] = o[k] * w[k];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    a[k] = e[k] + o[k];
    a[k + 8] = e[k] - o[k];
  }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(Cx<T>* a) {
  if constexpr (R == 2) dft2<T, INV>(a);
  else if constexpr (R == 3) dft3<T, INV>(a);
  else if constexpr (R == 4) dft4<T, INV>(a);
  else if constexpr (R == 8) dft8<T, INV>(a);
  else if constexpr (R == 16) dft16<T, INV>(a);
  else static_assert(R == 2, "unsupported radix");
}

// ------------------------------------------------------------------- stages
template <int L, int S>
struct FftSpan {  // product of the radices before stage S
  static constexpr int value = FftSpan<L, S - 1>::value * FftPlan<L>::R[S - 1];
};
template <int L>
struct FftSpan<L, 0> {
  static constexpr int value = 1;
};

// Element index held by register e of lane g at the first stage's input and
// the last stage's output.
template <int L>
__device__ __forceinline__ int fft_elem(int g, int e) {
  using P = FftPlan<L>;
  constexpr int R1 = P::R[0];
  return g + P::G * (e / R1) + (e % R1) * (L / R1);
}

// Twiddle table: w_{2L}^t = exp(-2 pi i t / (2L)) for t < L, stored at LDS
// slot lds_pad(t) (the padding spreads the strided stage-twiddle reads over
// the banks); the other half follows from w_{2L}^{t+L} = -w_{2L}^t.
template <typename T, int L>
__device__ __forceinline__ Cx<T> tw_2l(const Cx<T>* __restrict__ tw, int t) {
  const bool hi = t >= L;
  const Cx<T> w = tw[lds_pad(hi ? t - L : t)];
  return hi ? Cx<T>{-w.re, -w.im} : w;
}

// w_{2L}^t for t < L
template <typename T, int L>
__device__ __forceinline__ Cx<T> tw_lo(const Cx<T>* __restrict__ tw, int t) {
  return tw[lds_pad(t)];
}

// Copy the L-entry twiddle table into LDS (lds_len<L>() slots; whole
// workgroup; caller syncs).
template <typename T, int L>
__device__ __forceinline__ void stage_twiddles(Cx<T>* __restrict__ dst, const Cx<T>* __restrict__ src) {
  for (int t = threadIdx.x; t < L; t += blockDim.x) dst[lds_pad(t)] = src[t];
}

template <typename T, int L, bool INV, int S>
struct FftStage {
  using P = FftPlan<L>;
  static constexpr int R = P::R[S];
  static constexpr int Ns = FftSpan<L, S>::value;
  static constexpr int E = P::E;
  static constexpr int U = E / R;

  __device__ __forceinline__ static void run(Cx<T> (&v)[E], int g, Cx<T>* __restrict__ buf,
                                             const Cx<T>* __restrict__ tw2) {
    // twiddle and butterfly
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (Ns > 1) {
        const int b = g + P::G * u;
        const int j = b % Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          Cx<T> w = tw_2l<T, L>(tw2, 2 * (r * j * (L / (Ns * R))));
          if constexpr (INV) w.im = -w.im;
          v[u * R + r] = v[u * R + r] * w;
        }
      }
      dft<T, R, INV>(&v[u * R]);
    }
    if constexpr (S + 1 < P::NST) {
      constexpr int Rn = P::R[S + 1];
      constexpr int Un = E / Rn;
      wave_sync();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int b = g + P::G * u;
        const int base = (b / Ns) * Ns * R + (b % Ns);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[lds_pad(base + r * Ns)] = v[u * R + r];
      }
      wave_sync();
#pragma unroll
      for (int u = 0; u < Un; ++u) {
        const int b = g + P::G * u;
#pragma unroll
        for (int r = 0; r < Rn; ++r) v[u * Rn + r] = buf[lds_pad(b + r * (L / Rn))];
      }
      FftStage<T, L, INV, S + 1>::run(v, g, buf, tw2);
    }
  }
};

// In-register FFT of length L: v holds element fft_elem<L>(g, e) in register e
// on entry and the transform at the same elements on exit.  buf is this
// group's LDS exchange area of lds_len<L>() elements.
template <typename T, int L, bool INV>
__device__ __forceinline__ void fft_regs(Cx<T> (&v)[FftPlan<L>::E], int g, Cx<T>* __restrict__ buf,
                                         const Cx<T>* __restrict__ tw2) {
  FftStage<T, L, INV, 0>::run(v, g, buf, tw2);
}

// Two independent FFTs of length L interleaved stage by stage in one group
// (separate exchange buffers; each twiddle is loaded once for both), which
// doubles the independent work available between LDS round trips.
template <typename T, int L, bool INV, int S>
struct FftStage2 {
  using P = FftPlan<L>;
  static constexpr int R = P::R[S];
  static constexpr int Ns = FftSpan<L, S>::value;
  static constexpr int E = P::E;
  static constexpr int U = E / R;

  __device__ __forceinline__ static void run(Cx<T> (&a)[E], Cx<T> (&b)[E], int g, Cx<T>* __restrict__ bufa,
                                             Cx<T>* __restrict__ bufb, const Cx<T>* __restrict__ tw2) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (Ns > 1) {
        const int bb = g + P::G * u;
        const int j = bb % Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          Cx<T> w = tw_2l<T, L>(tw2, 2 * (r * j * (L / (Ns * R))));
          if constexpr (INV) w.im = -w.im;
          a[u * R + r] = a[u * R + r] * w;
          b[u * R + r] = b[u * R + r] * w;
        }
      }
      dft<T, R, INV>(&a[u * R]);
      dft<T, R, INV>(&b[u * R]);
    }
    if constexpr (S + 1 < P::NST) {
      constexpr int Rn = P::R[S + 1];
      constexpr int Un = E / Rn;
      wave_sync();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int bb = g + P::G * u;
        const int base = (bb / Ns) * Ns * R + (bb % Ns);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          bufa[lds_pad(base + r * Ns)] = a[u * R + r];
          bufb[lds_pad(base + r * Ns)] = b[u * R + r];
        }
      }
      wave_sync();
#pragma unroll
      for (int u = 0; u < Un; ++u) {
        const int bb = g + P::G * u;
#pragma unroll
        for (int r = 0; r < Rn; ++r) {
          a[u * Rn + r] = bufa[lds_pad(bb + r * (L / Rn))];
          b[u * Rn + r] = bufb[lds_pad(bb + r * (L / Rn))];
        }
      }
      FftStage2<T, L, INV, S + 1>::run(a, b, g, bufa, bufb, tw2);
    }
  }
};

template <typename T, int L, bool INV>
__device__ __forceinline__ void fft2_regs(Cx<T> (&a)[FftPlan<L>::E], Cx<T> (&b)[FftPlan<L>::E], int g,
                                          Cx<T>* __restrict__ bufa, Cx<T>* __restrict__ bufb,
                                          const Cx<T>* __restrict__ tw2) {
  FftStage2<T, L, INV, 0>::run(a, b, g, bufa, bufb, tw2);
}
