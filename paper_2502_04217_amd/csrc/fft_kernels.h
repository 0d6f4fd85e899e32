// Pencil-FFT kernel templates shared by the FFT drivers: fft.hip
// instantiates them for power-of-two pencil lengths, fft_mixed_f64.hip and
// fft_mixed_f32.hip for lengths with odd factors 3, 5 and 7 (the
// non-power-of-two grids of the paper's synthetic size table, small grids
// that exercise each radix, and odd extents on axes 1 and 2); fft_any.hip
// serves the other lengths 2^a 3^b 5^c 7^d up to 1024 through the same
// helpers.
//
// Each pencil FFT is a Stockham sequence of radix-r stages: the first stage
// reads its inputs straight from global memory into registers, intermediate
// stages exchange through LDS, and the last stage writes from registers to
// global memory (or into an epilogue).  A stage of radix r has L/r
// butterflies; the NT threads of a pencil take butterflies j = t + i*NT.
// When NT divides L/r every thread has the same number of butterflies;
// otherwise (an odd radix that does not divide the per-thread element count)
// the stage is guarded, and the spare register slots of the last round go
// unused.
#pragma once

#include "csipm_internal.h"

#include <type_traits>

namespace csipm {
namespace fftk {

constexpr int kLdsBytes = 65536;     // LDS budget of an axis-3 workgroup

// ------------------------------------------------------------- radix plan --
constexpr int odd_part(int x) {
  while (x > 0 && x % 2 == 0) x /= 2;
  return x;
}
constexpr int smallest_odd_factor(int x) {
  for (int p = 3; p <= x; p += 2)
    if (x % p == 0) return p;
  return x;
}
// k-th odd prime factor of F (ascending, with multiplicity)
constexpr int odd_factor(int F, int k) {
  int p = smallest_odd_factor(F);
  for (int i = 0; i < k; ++i) {
    F /= p;
    p = smallest_odd_factor(F);
  }
  return p;
}
constexpr int odd_factor_count(int F) {
  int c = 0;
  while (F > 1) {
    F /= smallest_odd_factor(F);
    ++c;
  }
  return c;
}

// Stage plan of a length-L pencil with E elements per thread (NT = L/E
// threads).  The power-of-two part of L is split into stages of radix P2
// (the power-of-two part of E; 4 when E is odd) and one remainder stage;
// the odd prime factors of L follow as stages of their own.
template <int L, int E>
struct Radix {
  static_assert(L % E == 0, "elements per thread must divide the pencil length");
  static constexpr int NT = L / E;
  static constexpr int LP = L / odd_part(L);
  static constexpr int P2 = (E / odd_part(E)) > 1 ? E / odd_part(E) : (LP < 4 ? LP : 4);
  static constexpr int nfull() {
    int c = 0, r = LP;
    while (P2 > 1 && r >= P2) { r /= P2; ++c; }
    return c;
  }
  static constexpr int NFULL = nfull();
  static constexpr int rem() {
    int r = LP;
    for (int i = 0; i < NFULL; ++i) r /= P2;
    return r;
  }
  static constexpr int REM = rem();
  static constexpr int NPOW = NFULL + (REM > 1 ? 1 : 0);
  // a length-1 pencil (a 2D or 1D grid) has one identity stage of radix 1
  static constexpr int NSTAGES = L == 1 ? 1 : NPOW + odd_factor_count(odd_part(L));
  static constexpr int radix(int s) {
    return L == 1 ? 1 : (s < NFULL ? P2 : (s < NPOW ? REM : odd_factor(odd_part(L), s - NPOW)));
  }
  static constexpr int ns(int s) {
    int v = 1;
    for (int i = 0; i < s; ++i) v *= radix(i);
    return v;
  }
  // butterflies per thread in stage s, and whether every one is real
  static constexpr int nb(int s) { return (L / radix(s) + NT - 1) / NT; }
  static constexpr bool exact(int s) { return (L / radix(s)) % NT == 0; }
  static constexpr int vmax() {
    int m = 0;
    for (int s = 0; s < NSTAGES; ++s) m = nb(s) * radix(s) > m ? nb(s) * radix(s) : m;
    return m;
  }
  static constexpr int VMAX = vmax();   // register slots per thread
};

// cos and sin of 2 pi m / R for the odd radices (folded to literals once
// the butterfly loops are unrolled)
__host__ __device__ constexpr double root_cos(int R, int m) {
  const int k = m % R;
  const int a = 2 * k <= R ? k : R - k;
  if (a == 0) return 1.0;
  if (R == 3) return -0.5;
  if (R == 5) return a == 1 ? 0.30901699437494742410 : -0.80901699437494742410;
  return a == 1 ? 0.62348980185873353053 : (a == 2 ? -0.22252093395631440429 : -0.90096886790241912624);
}
__host__ __device__ constexpr double root_sin(int R, int m) {
  const int k = m % R;
  const bool neg = 2 * k > R;
  const int a = neg ? R - k : k;
  double v = 0.0;
  if (a != 0) {
    if (R == 3) v = 0.86602540378443864676;
    else if (R == 5) v = a == 1 ? 0.95105651629515357212 : 0.58778525229247312917;
    else v = a == 1 ? 0.78183148246802980871 : (a == 2 ? 0.97492791218182360702 : 0.43388373911755812048);
  }
  return neg ? -v : v;
}

// In-register DFT of odd size R in natural order, out[k] = sum_j v[j]
// exp(DIR 2 pi i j k / R), from the conjugate-pair split: with a_j = v_j +
// v_{R-j} and b_j = v_j - v_{R-j} (j = 1..(R-1)/2),
//   out[k] = v_0 + sum_j a_j cos(2 pi jk/R) + DIR i sum_j b_j sin(2 pi jk/R),
// and out[R-k] the same with the sine sum negated.
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_odd(cx<T>* v) {
  static_assert(R == 3 || R == 5 || R == 7, "odd radices 3, 5 and 7");
  constexpr int H = (R - 1) / 2;
  cx<T> a[H], b[H];
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    a[j - 1] = cadd(v[j], v[R - j]);
    b[j - 1] = csub(v[j], v[R - j]);
  }
  cx<T> out[R];
  out[0] = v[0];
#pragma unroll
  for (int j = 0; j < H; ++j) out[0] = cadd(out[0], a[j]);
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    cx<T> x = v[0], y = {T(0), T(0)};
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const T c = T(root_cos(R, j * k)), s = T(root_sin(R, j * k));
      x = {x.re + a[j - 1].re * c, x.im + a[j - 1].im * c};
      y = {y.re + b[j - 1].re * s, y.im + b[j - 1].im * s};
    }
    const cx<T> iy = cmul_i<DIR>(y);
    out[k] = cadd(x, iy);
    out[R - k] = csub(x, iy);
  }
#pragma unroll
  for (int k = 0; k < R; ++k) v[k] = out[k];
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_any(cx<T>* v) {
  if constexpr ((R & (R - 1)) == 0) dft_reg<R, DIR, T>(v);
  else dft_odd<R, DIR, T>(v);
}

template <typename T, typename Tw>
__device__ __forceinline__ cx<T> twiddle(const Tw* tw, int idx, int dir) {
  cx<T> w = tw[idx];
  if (dir > 0) w.im = -w.im;
  return w;
}

// Calls f(slot, element) for the inputs of stage S (element j + q L/r of
// butterfly j), which are also the outputs of the last stage; slot i*r + q
// of the register block holds value q of the thread's i-th butterfly.
template <int L, int E, int S, class F>
__device__ __forceinline__ void for_stage_io(int t, F f) {
  using RP = Radix<L, E>;
  constexpr int r = RP::radix(S);
  constexpr int NB = RP::nb(S);
  constexpr bool EX = RP::exact(S);
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + i * RP::NT;
    if (EX || j < L / r) {
#pragma unroll
      for (int q = 0; q < r; ++q) f(i * r + q, j + q * (L / r));
    }
  }
}

// Applies stage S of a length-L Stockham FFT to the register block v.
template <typename T, int L, int E, int DIR, int S>
__device__ __forceinline__ void stage_compute(cx<T>* v, int t, const cx<T>* tw) {
  using RP = Radix<L, E>;
  constexpr int r = RP::radix(S);
  constexpr int Ns = RP::ns(S);
  constexpr int NT = RP::NT;
  constexpr int NB = RP::nb(S);
  constexpr bool EX = RP::exact(S);
  // Twiddles w^(jm q TS), jm = j mod Ns, of butterfly j = t + i NT: one
  // table load per butterfly, the higher powers w^q as products of lower
  // ones (w^2 = w w, w^3 = w w^2, w^4 = w^2 w^2, ...; depth log2 r).  Where
  // NT is a multiple of Ns every butterfly of the thread has jm = t mod Ns,
  // and one set serves them all; where L / r <= Ns every one has jm = j, and
  // w^(j TS) = w^(t TS) w^(i NT TS): one load per thread and a uniform factor
  // (a scalar load) per further butterfly.  Table loads were the pencil
  // passes' most frequent vector-memory instruction and held the most
  // registers.
  constexpr int TS = L / (Ns * r);
  constexpr bool SHARED = Ns > 1 && NB > 1 && NT % Ns == 0;
  constexpr bool LASTJ = Ns > 1 && NB > 1 && !SHARED && L / r <= Ns;
  auto powers = [](cx<T>* wq) {
#pragma unroll
    for (int q = 2; q < r; ++q) {
      const int hb = 1 << (31 - __builtin_clz(q));
      wq[q] = q == hb ? cmul(wq[hb / 2], wq[hb / 2]) : cmul(wq[q - hb], wq[hb]);
    }
  };
  cx<T> ws[SHARED ? r : 1];
  if constexpr (SHARED) {
    ws[1] = twiddle<T>(tw, (t % Ns) * TS, DIR);
    powers(ws);
  }
  cx<T> wt{T(1), T(0)};
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + i * NT;
    if (EX || j < L / r) {
      if constexpr (Ns > 1) {
        if constexpr (SHARED) {
#pragma unroll
          for (int q = 1; q < r; ++q) v[i * r + q] = cmul(v[i * r + q], ws[q]);
        } else {
          cx<T> wq[r];
          if constexpr (LASTJ) {
            if (i == 0) wt = twiddle<T>(tw, t * TS, DIR);
            wq[1] = i == 0 ? wt : cmul(wt, twiddle<T>(tw, i * NT * TS, DIR));
          } else {
            wq[1] = twiddle<T>(tw, (j % Ns) * TS, DIR);
          }
          powers(wq);
#pragma unroll
          for (int q = 1; q < r; ++q) v[i * r + q] = cmul(v[i * r + q], wq[q]);
        }
      }
      dft_any<r, DIR, T>(&v[i * r]);
    }
  }
}

// Writes stage S outputs to LDS (Stockham destination index) and reads
// stage S+1 inputs back.  `lidx(e)` maps a pencil element to its LDS slot.
template <typename T, int L, int E, int S, class LIdx>
__device__ __forceinline__ void stage_exchange(cx<T>* v, int t, cx<T>* lds, LIdx lidx) {
  using RP = Radix<L, E>;
  constexpr int r = RP::radix(S);
  constexpr int Ns = RP::ns(S);
  constexpr int NT = RP::NT;
  constexpr int NB = RP::nb(S);
  constexpr bool EX = RP::exact(S);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + i * NT;
    if (EX || j < L / r) {
      const int base = (j / Ns) * Ns * r + (j % Ns);
#pragma unroll
      for (int q = 0; q < r; ++q) lds[lidx(base + q * Ns)] = v[i * r + q];
    }
  }
  __syncthreads();
  for_stage_io<L, E, S + 1>(t, [&](int slot, int e) { v[slot] = lds[lidx(e)]; });
}

// Runs all stages; inputs in the first-stage pattern, outputs left in
// registers in the last-stage pattern (both as for_stage_io lists them).
template <typename T, int L, int E, int DIR, int S, class LIdx>
__device__ __forceinline__ void fft_stages(cx<T>* v, int t, cx<T>* lds, LIdx lidx, const cx<T>* tw) {
  using RP = Radix<L, E>;
  stage_compute<T, L, E, DIR, S>(v, t, tw);
  if constexpr (S + 1 < RP::NSTAGES) {
    stage_exchange<T, L, E, S>(v, t, lds, lidx);
    fft_stages<T, L, E, DIR, S + 1>(v, t, lds, lidx, tw);
  }
}

template <int L, int E>
constexpr int last_stage() { return Radix<L, E>::NSTAGES - 1; }

// Elements per thread of a pencil with odd factors: the odd part (its
// smallest prime factor when the odd part exceeds 7) times up to 4: 12, 20
// or 28 values for odd parts 3, 5, 7; 20 for odd part 35 (70, 280, 560),
// whose largest radix-7 stage is then the only guarded one.
constexpr int mixed_e(int L) {
  const int F = odd_part(L), P = L / F;
  const int f = F <= 7 ? F : smallest_odd_factor(F);
  return f * (P < 4 ? P : 4);
}
constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }

// ------------------------------------------------------- block reduction --

// Block sums of NQ values; thread 0 writes out[q * stride + blockIdx.x].
// `red` is LDS scratch of at least NQ * NTHREADS/64 doubles; it may alias the
// FFT exchange buffer, so the block synchronises before writing it.
// The last NMAX quantities are maxima (of non-negative values), the others sums.
template <int NTHREADS, int NQ, int NMAX = 0>
__device__ __forceinline__ void block_sums_store(const double* v, double* out, int stride, double* red) {
  static_assert(NTHREADS % 64 == 0, "block reductions need whole waves");
  constexpr int NW = NTHREADS / 64;
  double w[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) w[q] = q >= NQ - NMAX ? wave_max(v[q]) : wave_sum(v[q]);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[q * NW + wv] = w[q];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double a = 0.0;
      for (int i = 0; i < NW; ++i) a = q >= NQ - NMAX ? fmax(a, red[q * NW + i]) : a + red[q * NW + i];
      out[q * stride + blockIdx.x] = a;
    }
}

// ------------------------------------------------------------ epilogues --
// Applied to each output element h = (H p)[idx] of the last forward pass
// (the m = 0 plane by the workgroups that unmix it).
struct EpiNone {
  static constexpr int NRED = 0;
  static constexpr int NMAX = 0;
  static constexpr bool PRO = false;
  double* partial = nullptr;
  int pstride = 0;
};

// Plain output with the fused CG direction update on input (axis-1 inverse
// pass of K p): p <- z + beta p as p is loaded, written back to p outside
// the m = 0 plane (there the K epilogue writes it).  z null: no update.
template <typename T>
struct EpiP {
  static constexpr int NRED = 0;
  static constexpr int NMAX = 0;
  static constexpr bool PRO = true;
  cx<T>* p;
  const cx<T>* z;
  const double* beta;
  double* partial = nullptr;
  int pstride = 0;
};

// q = K p (equation "condensedkkt" in Sigma form) and p.q
template <typename T>
struct EpiK {
  static constexpr int NRED = 1;
  static constexpr int NMAX = 0;
  static constexpr bool PRO = false;
  KArgs<T> a;
  double* partial;
  int pstride;
  // (m0: an element of the m = 0 plane, whose p_beta the inverse pass did
  // not update)
  __device__ __forceinline__ void operator()(long long idx, cx<T> h, double* acc, bool m0) const {
    cx<T> pb = reinterpret_cast<const cx<T>*>(a.pb)[idx];
    cx<T> pz = reinterpret_cast<const cx<T>*>(a.pz)[idx];
    if (a.u.zb) {   // fused direction update of p_z (p_beta was updated on input)
      const T be = (T)*a.u.beta;
      if (m0) {
        const cx<T> zb = reinterpret_cast<const cx<T>*>(a.u.zb)[idx];
        pb = {zb.re + be * pb.re, zb.im + be * pb.im};
        reinterpret_cast<cx<T>*>(a.u.pb)[idx] = pb;
      }
      const cx<T> zz = reinterpret_cast<const cx<T>*>(a.u.zz)[idx];
      pz = {zz.re + be * pz.re, zz.im + be * pz.im};
      reinterpret_cast<cx<T>*>(a.u.pz)[idx] = pz;
    }
    const cx<T> s1 = reinterpret_cast<const cx<T>*>(a.sig1)[idx];
    const cx<T> s2 = reinterpret_cast<const cx<T>*>(a.sig2)[idx];
    cx<T> qb, qz;
    k_block<T>(h.re, pb.re, pz.re, s1.re, s2.re, qb.re, qz.re);
    k_block<T>(h.im, pb.im, pz.im, s1.im, s2.im, qb.im, qz.im);
    reinterpret_cast<cx<T>*>(a.qb)[idx] = qb;
    reinterpret_cast<cx<T>*>(a.qz)[idx] = qz;
    acc[0] += (double)pb.re * (double)qb.re + (double)pb.im * (double)qb.im + (double)pz.re * (double)qz.re +
              (double)pz.im * (double)qz.im;
  }
};

// FP64 refinement residual r = h - K d: writes H d_beta (the transform output
// itself), sums r.P_c^{-1}r and takes max |r|.  A further inner solve, when
// one is needed, builds its FP32 start from H d_beta elementwise
// (k_ref_restart).
struct EpiR {
  static constexpr int NRED = 2;
  static constexpr int NMAX = 1;
  static constexpr bool PRO = false;
  RArgs a;
  double* partial;
  int pstride;
  __device__ __forceinline__ void operator()(long long idx, cx<double> h, double* acc, bool) const {
    using D2 = cx<double>;
    const D2 db = reinterpret_cast<const D2*>(a.db)[idx], dz = reinterpret_cast<const D2*>(a.dz)[idx];
    const D2 s1 = reinterpret_cast<const D2*>(a.sig1)[idx], s2 = reinterpret_cast<const D2*>(a.sig2)[idx];
    const D2 hb = reinterpret_cast<const D2*>(a.hb)[idx], hz = reinterpret_cast<const D2*>(a.hz)[idx];
    const float2 c = a.c ? reinterpret_cast<const float2*>(a.c)[idx] : make_float2(1.0f, 1.0f);
    reinterpret_cast<D2*>(a.hd)[idx] = h;
    const double hv[2] = {h.re, h.im}, dbv[2] = {db.re, db.im}, dzv[2] = {dz.re, dz.im}, g1[2] = {s1.re, s1.im},
                 g2[2] = {s2.re, s2.im}, rhb[2] = {hb.re, hb.im}, rhz[2] = {hz.re, hz.im}, cv[2] = {c.x, c.y};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      double qb, qz, zb, zz;
      k_block<double>(hv[k], dbv[k], dzv[k], g1[k], g2[k], qb, qz);
      const double rb = rhb[k] - qb, rz = rhz[k] - qz;
      pinv_block(rb, rz, g1[k], g2[k], cv[k], zb, zz);
      acc[0] += rb * zb + rz * zz;
      acc[1] = fmax(acc[1], fmax(fabs(rb), fabs(rz)));
    }
  }
};

// --------------------------------------------------- strided pencil pass --
// Complex FFT along axis 1 or 2 over the array [N1][N2][M].  Pencil q has
// base offset (q / inner) * outer + q % inner and element stride estride.
template <typename T>
struct StridedGeom {
  int inner;
  long long outer;
  long long estride;
  int batch;
};

// Tile shape of the strided (axis-1/2) passes per complex size w in bytes,
// pencil length L, axis and direction: elements per thread E and pencils
// per workgroup TM (LDS = TM L w, at most 1024 threads, TM a power of two).
// Power-of-two pencils, chosen from measurements at 256^3: 8 elements per
// thread for the FP64 axis-2 passes and the FP32 axis-1 forward pass, 16
// otherwise; 128 KB tiles for axis 1 except the FP64 inverse pass (64 KB),
// 64 KB for axis 2.  Pencils with odd factors take mixed_e elements.
constexpr int strided_e(int w, int L, int axis, int dir) {
  if (odd_part(L) != 1) return mixed_e(L);
  const int e = ((w == 16 && axis == 2) || (w == 8 && axis == 1 && dir < 0) ||
                   (w == 16 && axis == 1 && dir > 0 && L >= 512))
                    ? 8 : 16;
  return L < e ? L : e;
}
constexpr int strided_lds(int w, int axis, int dir, int L) {
  return axis == 2 ? 65536 : (w == 16 && dir > 0 && L < 512 ? 65536 : 131072);
}
// TM is the power of two that the LDS budget gives (at most 64), raised
// until each access is a run of at least 128 contiguous bytes (a whole
// cache line) and the workgroup is whole waves (block reductions), within
// 160 KB of LDS and 1024 threads.
constexpr int strided_tm(int w, int L, int axis, int dir) {
  const int nt = L / strided_e(w, L, axis, dir);
  int tm = strided_lds(w, axis, dir, L) / (L * w);
  if (tm > 64) tm = 64;
  if (tm < 1) tm = 1;
  int p = 1;
  while (2 * p <= tm) p *= 2;
  tm = p;
  while (tm * w < 128 && 2 * tm * L * w <= 163840 && 2 * tm * nt <= 1024) tm *= 2;
  while ((tm * nt) % 64 != 0 && 2 * tm * L * w <= 163840 && 2 * tm * nt <= 1024) tm *= 2;
  while (tm * nt > 1024) tm >>= 1;
  return tm;
}
template <typename T, int L, int AX, int DIR>
constexpr int strided_threads() {
  constexpr int w = int(sizeof(cx<T>));
  return strided_tm(w, L, AX, DIR) * (L / strided_e(w, L, AX, DIR));
}

// ------------------------------------------------ the m = 0 plane (axis 1) --
// In the m = 0 plane the internal layout holds the two self-paired planes
// k3 = 0 and k3 = N3/2 of the real parametrisation, whose coefficients pair
// (k1, k2) with (-k1, -k2) (derivation "map"): the spectrum U the inverse
// transform needs at (k1, k2, 0) mixes the stored values W of both, and the
// forward transform's output H is unmixed the same way.  In an axis-1 pass
// the lane of pencil (k2, m = 0) also reads the pencil of the partner row
// (N2 - k2) mod N2 at the reversed index -k1:
//   inverse: U = W on self-conjugate (k1, k2), (W + i W(-k)) / sqrt2 on a
//            canonical one, (W(-k) - i W) / sqrt2 on its mirror, formed as
//            the two rows are read;
//   forward: with F the FFT along k1 and R the reversal j1 -> -j1 (so that
//            F(R b)(k1) = F(b)(-k1)), the unmixed output of a canonical row
//            a paired with row b is F((a + R b) / sqrt2) and that of the
//            mirror row b is F(i (b - R a) / sqrt2): the unmixing is applied
//            to the inputs.  A self-paired row (k2 = 0 or N2/2) is both, so
//            the forward pass gives it two lanes of one workgroup at the
//            front of the grid: one transforms (a + R a) / sqrt2 and writes
//            the canonical and (scaled by 1/sqrt2) self-conjugate elements,
//            the other i (a - R a) / sqrt2 and writes the mirror elements.
// With the fused CG direction update the m = 0 lanes of the inverse pass
// read p but do not write it back (a partner row may still need the old
// value); the forward pass's K epilogue updates p_beta there instead.
// 2D class of (k1, k2): 0 self-conjugate, 1 canonical, 2 the mirror of a
// canonical index.
__host__ __device__ __forceinline__ int cls2(int k1, int k2, int n1, int n2) {
  const bool e1 = (2 * k1 == n1) || k1 == 0;
  const bool e2 = (2 * k2 == n2) || k2 == 0;
  if (e1 && e2) return 0;
  if (2 * k2 < n2 && k2 >= 1) return 1;
  if (e2 && k1 >= 1 && 2 * k1 < n1) return 1;
  return 2;
}
__host__ __device__ __forceinline__ bool self_paired_row(int k2, int n2) { return k2 == 0 || 2 * k2 == n2; }
// lane li of the forward pass's first workgroup: the two self-paired rows,
// each on a canonical (even li) and a mirror (odd li) lane; -1: idle
__host__ __device__ __forceinline__ int plane0_self_row(int li, int n2) {
  if (li < 2) return 0;
  if (li < 4) return (n2 % 2 == 0 && n2 >= 2) ? n2 / 2 : -1;
  return -1;
}
struct Plane0 {
  int n2;           // N2
  int ndedicated;   // workgroups in front of the tiles (forward axis-1 pass: 1)
};

// The pencil a lane of a strided pass transforms (pencil p of the
// workgroup's TM) and its part in the m = 0 plane (axis 1).
struct Lane12 {
  long long base;   // offset of the pencil's element 0
  int k2;           // row of an m = 0 lane
  bool active;      // the lane has a pencil
  bool m0;          // the pencil lies in the m = 0 plane
  bool canon;       // an m = 0 lane of a canonical row (or the even lane of a self-paired one)
  bool ded;         // the workgroup of the self-paired rows (forward axis-1 pass)
};
template <int AX, int DIR, typename T>
__device__ __forceinline__ Lane12 lane12(int p, int TM, const StridedGeom<T>& geo, int m, const Plane0& pl) {
  constexpr bool MIX = AX == 1;
  Lane12 ln;
  ln.ded = MIX && DIR < 0 && (int)blockIdx.x < pl.ndedicated;
  ln.k2 = 0;
  ln.canon = true;
  ln.m0 = false;
  int qpen;
  if (MIX && ln.ded) {
    ln.k2 = plane0_self_row(p, pl.n2);
    ln.active = ln.k2 >= 0;
    ln.m0 = true;
    ln.canon = (p & 1) == 0;
    qpen = ln.active ? ln.k2 * m : 0;
  } else {
    qpen = ((int)blockIdx.x - (MIX ? pl.ndedicated : 0)) * TM + p;
    ln.active = qpen < geo.batch;
    if (MIX && ln.active && qpen % m == 0) {
      ln.m0 = true;
      ln.k2 = qpen / m;
      ln.canon = 2 * ln.k2 < pl.n2;
      if (DIR < 0 && self_paired_row(ln.k2, pl.n2)) ln.active = false;   // (taken by the first workgroup)
    }
  }
  ln.base = ln.active ? (long long)(qpen / geo.inner) * geo.outer + (qpen % geo.inner) : 0;
  return ln;
}

// The partner rows of the workgroup's m = 0 lanes, reversed (element e of
// slot r holds element -e of slot r's partner row; with the direction
// update applied), staged in lds by all nthr threads, so that each thread
// loads at most a few of them instead of the m = 0 lanes each waiting on a
// row of scattered loads.  Slot r holds the partner of row first + r, for
// the rows whose m = 0 pencil falls in the tile (pencils q0 .. q0 + TM - 1);
// in the forward pass's first workgroup lanes 0-3 are the slots (partner =
// own row).  Returns the slot count (uniform over the workgroup; 0: no
// m = 0 lane, nothing staged and no barrier) and the lane's slot.
template <typename T, int DIR, class Epi>
__device__ __forceinline__ int stage_partners(cx<T>* lds, const cx<T>* src, int L, int TM, int nthr,
                                              const StridedGeom<T>& geo, int m, const Plane0& pl, const Epi& epi,
                                              bool upd, T be, bool ded, int p, int& slot) {
  const int q0 = ded ? 0 : ((int)blockIdx.x - pl.ndedicated) * TM;
  const int first = ded ? 0 : (q0 + m - 1) / m;
  const int nslot = ded ? 4 : (q0 + TM - 1) / m + 1 - first;
  slot = ded ? p : (q0 + p) / m - first;
  if (nslot <= 0) return nslot;
  for (int j = threadIdx.x; j < nslot * L; j += nthr) {
    const int r = j / L, i = j % L;
    int row;
    if (ded) {
      row = plane0_self_row(r, pl.n2);
    } else {
      row = first + r;
      if (row >= pl.n2 || (DIR < 0 && self_paired_row(row, pl.n2))) row = -1;
    }
    // (each branch stores its own value: a value merged across the branches
    // was kept in scratch memory)
    if (row >= 0) {
      const int prow = ded ? row : (pl.n2 - row) % pl.n2;
      const long long i1 = (long long)prow * m + (long long)((L - i) % L) * geo.estride;
      cx<T> y = src[i1];
      if constexpr (Epi::PRO) {
        if (upd) {
          const cx<T> zb = epi.z[i1];
          y = {zb.re + be * y.re, zb.im + be * y.im};
        }
      }
      lds[j] = y;
    } else {
      lds[j] = cx<T>{T(0), T(0)};
    }
  }
  __syncthreads();
  return nslot;
}

// Element e of an m = 0 lane's pencil x mixed with its staged partner y:
// on the inverse pass's input (U from the stored W), or the forward pass's
// unmixing applied to its input.
template <typename T, int DIR>
__device__ __forceinline__ cx<T> plane0_mix(cx<T> x, cx<T> y, int e, const Lane12& ln, int L, int n2) {
  const T rs2 = T(0.70710678118654752440);
  if constexpr (DIR > 0) {
    const int c = cls2(e, ln.k2, L, n2);
    return c == 0 ? x : (c == 1 ? cscale(cadd(x, cmul_i<1>(y)), rs2) : cscale(csub(y, cmul_i<1>(x)), rs2));
  } else {
    return ln.canon ? cscale(cadd(x, y), rs2) : cscale(cmul_i<1>(csub(x, y)), rs2);
  }
}

// Whether the lane writes output element e: the self-paired rows' lanes
// write the elements of their class (the self-conjugate ones scaled).
template <int AX, int DIR, typename T>
__device__ __forceinline__ bool plane0_keep(int e, cx<T>& h, const Lane12& ln, int L, int n2) {
  if (!(AX == 1 && DIR < 0 && ln.ded)) return true;
  const int c = cls2(e, ln.k2, L, n2);
  if (c == 0 && ln.canon) h = cscale(h, T(0.70710678118654752440));
  return ln.canon ? c != 2 : c == 2;
}

// Element idx of the input, with the fused direction update p <- z + beta p
// (written back outside the m = 0 plane: a partner row may still need the
// old value; the forward pass's K epilogue writes it).
template <typename T, class Epi>
__device__ __forceinline__ cx<T> load_input(const cx<T>* src, long long idx, bool active, bool upd, T be,
                                            const Epi& epi, bool keep_p) {
  cx<T> x = active ? src[idx] : cx<T>{T(0), T(0)};
  if constexpr (Epi::PRO) {
    if (upd && active) {
      const cx<T> zv = epi.z[idx];
      x = {zv.re + be * x.re, zv.im + be * x.im};
      if (!keep_p) epi.p[idx] = x;
    }
  }
  return x;
}

template <typename T, int L, int AX, int DIR, class Epi>
__global__ void __launch_bounds__((strided_threads<T, L, AX, DIR>()))
k_axis12(const cx<T>* src, cx<T>* dst, StridedGeom<T> geo,
         const cx<T>* __restrict__ tw, int m, Plane0 pl, Epi epi, const int* skip) {
  if (skip && *skip) return;
  constexpr int E = strided_e(int(sizeof(cx<T>)), L, AX, DIR);
  constexpr int TM = strided_tm(int(sizeof(cx<T>)), L, AX, DIR);
  constexpr int NT = L / E;
  constexpr int VM = Radix<L, E>::VMAX;
  constexpr int SL = last_stage<L, E>();
  constexpr bool MIX = AX == 1;
  static_assert(!MIX || TM >= 4, "the self-paired rows take four lanes of one workgroup");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int p = threadIdx.x % TM;
  const int t = threadIdx.x / TM;
  const Lane12 ln = lane12<AX, DIR>(p, TM, geo, m, pl);

  cx<T> v[VM];
  bool upd = false;
  T be = T(0);
  if constexpr (Epi::PRO) {
    upd = epi.z != nullptr;
    if (upd) be = (T)*epi.beta;
  }
  for_stage_io<L, E, 0>(t, [&](int s, int e) {
    v[s] = load_input(src, ln.base + (long long)e * geo.estride, ln.active, upd, be, epi, MIX && ln.m0);
  });
  // (the partner rows go to the tile's LDS, which the FFT stages do not use
  // before their first exchange, while the lanes' own loads are in flight)
  if constexpr (MIX) {
    int slot;
    if (stage_partners<T, DIR>(lds, src, L, TM, TM * NT, geo, m, pl, epi, upd, be, ln.ded, p, slot) > 0 &&
        ln.m0 && ln.active) {
      for_stage_io<L, E, 0>(t, [&](int s, int e) {
        v[s] = plane0_mix<T, DIR>(v[s], lds[slot * L + e], e, ln, L, pl.n2);
      });
    }
  }
  auto lidx = [p](int e) { return e * TM + p; };
  fft_stages<T, L, E, DIR, 0>(v, t, lds, lidx, tw);

  if constexpr (Epi::NRED > 0) {
    double acc[Epi::NRED];
#pragma unroll
    for (int q = 0; q < Epi::NRED; ++q) acc[q] = 0.0;
    if (ln.active) {
      for_stage_io<L, E, SL>(t, [&](int s, int e) {
        cx<T> h = v[s];
        if (plane0_keep<AX, DIR>(e, h, ln, L, pl.n2)) epi(ln.base + (long long)e * geo.estride, h, acc, MIX && ln.m0);
      });
    }
    block_sums_store<TM * NT, Epi::NRED, Epi::NMAX>(acc, epi.partial, epi.pstride,
                                                    reinterpret_cast<double*>(smem_raw));
  } else {
    if (ln.active) {
      for_stage_io<L, E, SL>(t, [&](int s, int e) {
        cx<T> h = v[s];
        if (plane0_keep<AX, DIR>(e, h, ln, L, pl.n2)) dst[ln.base + (long long)e * geo.estride] = h;
      });
    }
  }
}

// workgroups in front of the tiles of an axis-1 pass (the forward pass's
// workgroup of the self-paired rows)
inline int plane0_groups(int dir) { return dir < 0 ? 1 : 0; }

template <typename T, int L, int AX, int DIR, class Epi>
void launch_axis12_at(dim3 grid, const cx<T>* src, cx<T>* dst, StridedGeom<T> geo, const cx<T>* tw, int m,
                      int n2, Epi epi, const int* skip, hipStream_t s) {
  constexpr int TM = strided_tm(int(sizeof(cx<T>)), L, AX, DIR);
  constexpr int NT = L / strided_e(int(sizeof(cx<T>)), L, AX, DIR);
  static_assert((TM * NT) % 64 == 0 && TM * NT <= 1024, "strided tile must be whole waves");
  static_assert((size_t)TM * L * sizeof(cx<T>) <= 163840, "strided tile exceeds the LDS of a CU");
  const size_t shm = (size_t)TM * L * sizeof(cx<T>);
  const Plane0 pl{n2, AX == 1 ? plane0_groups(DIR) : 0};
  auto kern = k_axis12<T, L, AX, DIR, Epi>;
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL(kern, dim3(grid.x + pl.ndedicated), dim3(TM * NT), shm, s, src, dst, geo, tw, m, pl, epi, skip);
}

// ------------------------------------------------------ axis-3 (c2r/r2c) --
// Elements per thread of the axis-3 pass, the measured best per length:
// 8 for power-of-two pencils; for odd parts above 7 the smallest odd factor
// times up to 2 (10 at L = 280: 12 % and 17 % faster than 20 or 35 in FP32
// and FP64 at 256 x 256 x 560); mixed_e otherwise.
template <typename T>
constexpr int a3_e(int L) {
  if (odd_part(L) == 1) return L < 8 ? L : 8;
  if (odd_part(L) > 7) {
    const int P = L / odd_part(L);
    return smallest_odd_factor(odd_part(L)) * (P < 2 ? P : 2);
  }
  return mixed_e(L);
}
// one wave per workgroup: the pass synchronises between its many LDS
// stages, and at 256^3 the single-wave group is the fastest tile measured
// (4 pencils of 128 at 8 elements per thread)
constexpr int kA3Threads = 64;
template <typename T>
constexpr int a3_pad(int L) { return L + (L >= 16 ? L / 16 : 1); }
template <typename T>
constexpr int a3_pp(int L) {
  int nt = L / a3_e<T>(L);
  int pp = kA3Threads / nt;
  if (pp < 1) pp = 1;
  int lim = kLdsBytes / (a3_pad<T>(L) * int(sizeof(cx<T>)));
  while (pp > lim && pp > 1) pp >>= 1;
  return pp;
}

// The real transforms of length N3 = 2L through a half-length complex FFT
// (z_e = x[2e] + i x[2e+1]).  With the half spectrum X_e (e < L; X_0 packs
// the DC and Nyquist values as (re, im); the other coefficients carry the
// sqrt2 of the real parametrisation) and w = exp(-2 pi i e / N3):
// sqrt2 times the inverse transform's input is
// Z_e = X_e + conj X_{L-e} + i w* (X_e - conj X_{L-e}), with
// Z_0 = sqrt2 (X_0.re + X_0.im, X_0.re - X_0.im); from the forward half-length
// result Y, twice the half spectrum (the DC and Nyquist values once) is
// X_e = (Y_e + conj Y_{L-e}) - i w (Y_e - conj Y_{L-e}), with
// X_0 = (Y_0.re + Y_0.im, Y_0.re - Y_0.im).  These factors and the 1/sqrt(n)
// of each orthonormal transform are left to the one scale per output kind
// that the launch passes: a pass running both transforms multiplies once.
template <typename T>
__device__ __forceinline__ cx<T> c2r_dc(cx<T> x0) {
  const T s2 = T(1.41421356237309504880);
  return {(x0.re + x0.im) * s2, (x0.re - x0.im) * s2};
}
template <typename T>
__device__ __forceinline__ cx<T> c2r_pack(cx<T> xe, cx<T> xle, cx<T> w) {
  const cx<T> b = cconj(xle);
  const cx<T> sm = cadd(xe, b);
  const cx<T> d = csub(xe, b);
  w.im = -w.im;   // exp(+2 pi i e / N3)
  return cadd(sm, cmul_i<1>(cmul(w, d)));
}
template <typename T>
__device__ __forceinline__ cx<T> r2c_dc(cx<T> z0, T sc) { return {(z0.re + z0.im) * sc, (z0.re - z0.im) * sc}; }
template <typename T>
__device__ __forceinline__ cx<T> r2c_unpack(cx<T> a, cx<T> zle, cx<T> w, T sc) {
  const cx<T> b = cconj(zle);
  return cscale(cadd(cadd(a, b), cmul_i<-1>(cmul(w, csub(a, b)))), sc);
}
// z = (x[2e], x[2e+1]) with the unobserved samples zeroed: bits sh and
// sh + 1 of the mask word wd (the flat bit index of x[2e] is even, so both
// samples share a word)
template <typename T>
__device__ __forceinline__ cx<T> mask_pair(cx<T> z, uint32_t wd, int sh) {
  if (!((wd >> sh) & 1u)) z.re = T(0);
  if (!((wd >> (sh + 1)) & 1u)) z.im = T(0);
  return z;
}

// L = M = N3/2 complex values per pencil; pencil = (j1, j2).
template <typename T, int L, int MODE>
__global__ void __launch_bounds__(kA3Threads)
k_axis3(const cx<T>* src, cx<T>* dst, const uint32_t* __restrict__ mask,
        const cx<T>* __restrict__ twm, const cx<T>* __restrict__ tw3, int npencils, T sc_c2r,
        T sc_r2c_dc, T sc_r2c, const int* skip) {
  if (skip && *skip) return;
  constexpr int E = a3_e<T>(L);
  constexpr int NT = L / E;
  constexpr int PP = a3_pp<T>(L);
  static_assert(PP * NT <= kA3Threads, "axis-3 workgroup exceeds its launch bound");
  constexpr int LP = a3_pad<T>(L);
  constexpr int N3 = 2 * L;
  constexpr int VM = Radix<L, E>::VMAX;
  constexpr int SL = last_stage<L, E>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* ldsall = reinterpret_cast<cx<T>*>(smem_raw);
  const int p = threadIdx.x / NT;
  const int t = threadIdx.x % NT;
  const int pen = blockIdx.x * PP + p;
  const bool active = pen < npencils;
  const long long base = (long long)pen * L;
  cx<T>* lds = ldsall + p * LP;
  auto lidx = [](int e) { return e + (e >> 4); };

  cx<T> v[VM];
  if constexpr (MODE & A3_C2R) {
    // stage the packed half-spectrum through LDS: Z_e needs X_e and X_{L-e}
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int e = t + q * NT;
      lds[lidx(e)] = active ? src[base + e] : cx<T>{T(0), T(0)};
    }
    __syncthreads();
    // exp(-2 pi i e / N3) for e = t + k, k fixed by the unrolled slot:
    // tw3[t] (one load) times the uniform tw3[k] (a scalar load)
    const cx<T> w3t = tw3[t];
    for_stage_io<L, E, 0>(t, [&](int s, int e) {
      const int k = e - t;
      v[s] = e == 0 ? c2r_dc(lds[lidx(0)])
                    : c2r_pack(lds[lidx(e)], lds[lidx(L - e)], k == 0 ? w3t : cmul(w3t, tw3[k]));
    });
    fft_stages<T, L, E, +1, 0>(v, t, lds, lidx, twm);
    // z_e = x[2e] + i x[2e+1]
    // (a full pass leaves the inverse's scale to the forward output)
    for_stage_io<L, E, SL>(t, [&](int s, int e) {
      if constexpr (MODE == A3_FULL) {
        const long long bit = (long long)pen * N3 + 2 * e;
        v[s] = mask_pair(v[s], active ? mask[bit >> 5] : 0u, (int)(bit & 31));
      } else {
        v[s] = cscale(v[s], sc_c2r);
      }
    });
    if constexpr (MODE == A3_C2R) {
      if (active) for_stage_io<L, E, SL>(t, [&](int s, int e) { dst[base + e] = v[s]; });
      return;
    } else {
      // re-order to the first-stage pattern of the forward transform
      __syncthreads();
      for_stage_io<L, E, SL>(t, [&](int s, int e) { lds[lidx(e)] = v[s]; });
      __syncthreads();
      for_stage_io<L, E, 0>(t, [&](int s, int e) { v[s] = lds[lidx(e)]; });
    }
  } else {
    for_stage_io<L, E, 0>(t, [&](int s, int e) { v[s] = active ? src[base + e] : cx<T>{T(0), T(0)}; });
  }

  // forward half-length FFT of z' and the r2c post-processing
  int tf = t;
  if constexpr (MODE == A3_FULL && odd_part(L) > 1) {
    // the forward half recomputes its indices instead of keeping those of
    // the inverse half live across it
    asm volatile("" : "+v"(tf));
  }
  fft_stages<T, L, E, -1, 0>(v, tf, lds, lidx, twm);
  __syncthreads();
  for_stage_io<L, E, SL>(tf, [&](int s, int e) { lds[lidx(e)] = v[s]; });
  __syncthreads();
  if (!active) return;
  const cx<T> w3f = tw3[tf];
  for_stage_io<L, E, 0>(tf, [&](int s, int e) {
    const int k = e - tf;
    dst[base + e] = e == 0 ? r2c_dc(lds[lidx(0)], sc_r2c_dc)
                           : r2c_unpack(lds[lidx(e)], lds[lidx(L - e)], k == 0 ? w3f : cmul(w3f, tw3[k]), sc_r2c);
  });
}

template <typename T, int L>
void launch_axis3_at(int mode, int np, const cx<T>* cs, cx<T>* cd, const uint32_t* maskbits,
                     const cx<T>* twm, const cx<T>* tw3, T sc_c2r, T sc_dc, T sc_ac, const int* skip,
                     hipStream_t s) {
  constexpr int PP = a3_pp<T>(L);
  constexpr int NT = L / a3_e<T>(L);
  const size_t shm = (size_t)PP * a3_pad<T>(L) * sizeof(cx<T>);
  dim3 grid((np + PP - 1) / PP), block(PP * NT);
  if (shm > 65536) {
    (void)hipFuncSetAttribute((const void*)k_axis3<T, L, A3_FULL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shm);
    (void)hipFuncSetAttribute((const void*)k_axis3<T, L, A3_C2R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shm);
    (void)hipFuncSetAttribute((const void*)k_axis3<T, L, A3_R2C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shm);
  }
  if (mode == A3_FULL)
    hipLaunchKernelGGL((k_axis3<T, L, A3_FULL>), grid, block, shm, s, cs, cd, maskbits, twm, tw3, np, sc_c2r,
                       sc_dc, sc_ac, skip);
  else if (mode == A3_C2R)
    hipLaunchKernelGGL((k_axis3<T, L, A3_C2R>), grid, block, shm, s, cs, cd, maskbits, twm, tw3, np, sc_c2r,
                       sc_dc, sc_ac, skip);
  else
    hipLaunchKernelGGL((k_axis3<T, L, A3_R2C>), grid, block, shm, s, cs, cd, maskbits, twm, tw3, np, sc_c2r,
                       sc_dc, sc_ac, skip);
}

// ------------------------------------------------------- length dispatch --
// Grid extents with odd factors that have kernels (each as an axis-1/2
// pencil length N, and N/2 as the axis-3 half length): small grids that
// exercise radix 3, 5 and 7, and the non-power-of-two sizes of the paper's
// synthetic table (96, 192, 384, 560).
#define CSIPM_MIXED_LENGTHS(X) X(12) X(20) X(24) X(28) X(40) X(48) X(56) X(70) X(96) X(192) X(384) X(560)
// Odd extents, on axes 1 and 2 only (the odd-N case of the parametrisation:
// no Nyquist index on that axis); axis 3 keeps an even extent for its
// half-length transform.
#define CSIPM_ODD_LENGTHS(X) X(3) X(5) X(7) X(9) X(15) X(21) X(35) X(45)

// Launch a strided or axis-3 pass at a pencil length with odd factors;
// false when the length has no kernels.  Instantiated for FP64 in
// fft_mixed_f64.hip and for FP32 in fft_mixed_f32.hip.
template <typename T, int AX, int DIR, class Epi>
bool launch_axis12_mixed(int L, dim3 grid, const cx<T>* src, cx<T>* dst, StridedGeom<T> geo, const cx<T>* tw,
                         int m, int n2, Epi epi, const int* skip, hipStream_t s) {
#define CSIPM_A12(LL)                                                                     \
  case LL:                                                                                \
    launch_axis12_at<T, LL, AX, DIR, Epi>(grid, src, dst, geo, tw, m, n2, epi, skip, s); \
    return true;
  switch (L) {
    CSIPM_MIXED_LENGTHS(CSIPM_A12)
    CSIPM_ODD_LENGTHS(CSIPM_A12)
    default:
      return false;
  }
#undef CSIPM_A12
}

template <typename T>
bool launch_axis3_mixed(int L, int mode, int np, const cx<T>* cs, cx<T>* cd, const uint32_t* maskbits,
                        const cx<T>* twm, const cx<T>* tw3, T sc_c2r, T sc_dc, T sc_ac, const int* skip,
                        hipStream_t s) {
#define CSIPM_A3(NN)                                                                                     \
  case NN / 2:                                                                                           \
    launch_axis3_at<T, NN / 2>(mode, np, cs, cd, maskbits, twm, tw3, sc_c2r, sc_dc, sc_ac, skip, s); \
    return true;
  switch (L) {
    CSIPM_MIXED_LENGTHS(CSIPM_A3)
    default:
      return false;
  }
#undef CSIPM_A3
}

// Lengths with instantiated kernels: strided pencils (axes 1 and 2, and
// every axis of the odd-N3 transforms) and axis-3 half lengths.
inline bool templated12(int L) {
  if (L == 1 || L == 2 || (L >= 4 && L <= 1024 && (L & (L - 1)) == 0)) return true;
#define CSIPM_IS(NN) if (L == NN) return true;
  CSIPM_MIXED_LENGTHS(CSIPM_IS)
  CSIPM_ODD_LENGTHS(CSIPM_IS)
#undef CSIPM_IS
  return false;
}
inline bool templated3(int L) {
  if (L >= 2 && L <= 512 && (L & (L - 1)) == 0) return true;
#define CSIPM_IS(NN) if (2 * L == NN) return true;
  CSIPM_MIXED_LENGTHS(CSIPM_IS)
#undef CSIPM_IS
  return false;
}

// Every other length 2^a 3^b 5^c 7^d up to kAnyMaxLen: the passes with the
// pencils in LDS and a radix plan computed at launch (fft_any.hip).
constexpr int kAnyMaxLen = 1024;
struct AnyPlan {
  int L;        // pencil length
  int nst;      // stages
  int r[12];    // radix of each stage: 8, then 4 or 2, then 3, 5, 7
};
// false when L has a prime factor above 7 or lies outside [1, kAnyMaxLen]
bool any_plan(int L, AnyPlan& pl);
// pencils per workgroup at complex size w
int any_tm(int w, int L);
template <typename T, int AX, int DIR, class Epi>
bool launch_axis12_any(int L, dim3 grid, const cx<T>* src, cx<T>* dst, StridedGeom<T> geo, const cx<T>* tw, int m,
                       int n2, Epi epi, const int* skip, hipStream_t s);
template <typename T>
bool launch_axis3_any(int L, int mode, int np, const cx<T>* cs, cx<T>* cd, const uint32_t* maskbits,
                      const cx<T>* twm, const cx<T>* tw3, T sc_c2r, T sc_dc, T sc_ac, const int* skip,
                      hipStream_t s);
// pencils per workgroup of the strided pass that serves length L
inline int pass_tm(int w, int L, int axis, int dir) {
  return templated12(L) ? strided_tm(w, L, axis, dir) : any_tm(w, L);
}

// The instances used: PREFIX is empty where they are compiled and `extern`
// where they are only called.
#define CSIPM_MIXED_INST12(PREFIX, T, AX, DIR, EPI)                                                           \
  PREFIX template bool launch_axis12_mixed<T, AX, DIR, EPI>(int, dim3, const cx<T>*, cx<T>*, StridedGeom<T>, \
                                                            const cx<T>*, int, int, EPI, const int*, hipStream_t);
#define CSIPM_MIXED_INSTANCES(PREFIX, T)                                                                   \
  CSIPM_MIXED_INST12(PREFIX, T, 1, +1, EpiP<T>)                                                            \
  CSIPM_MIXED_INST12(PREFIX, T, 1, -1, EpiNone)                                                            \
  CSIPM_MIXED_INST12(PREFIX, T, 1, -1, EpiK<T>)                                                            \
  CSIPM_MIXED_INST12(PREFIX, T, 2, +1, EpiNone)                                                            \
  CSIPM_MIXED_INST12(PREFIX, T, 2, -1, EpiNone)                                                            \
  PREFIX template bool launch_axis3_mixed<T>(int, int, int, const cx<T>*, cx<T>*, const uint32_t*, const cx<T>*, \
                                             const cx<T>*, T, T, T, const int*, hipStream_t);

}  // namespace fftk
}  // namespace csipm
