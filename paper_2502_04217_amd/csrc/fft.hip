// Hand-written 3D real FFT passes for the operators A, A^T, H = A^T D A and
// the condensed KKT operator K (paper: "Matrix-free operators" and equation
// "condensedkkt").  gfx950, wave64.
//
// One apply of H is five volume passes over the n-real internal array plus
// two small passes over the plane m = 0:
//   premix   : m = 0 plane, real parametrisation -> spectrum (pairs k, -k)
//   axis 1   : inverse complex FFT along k1 (strided pencils)
//   axis 2   : inverse complex FFT along k2 (strided pencils)
//   axis 3   : c2r along k3, mask, r2c along k3 (contiguous pencils), using
//              a half-length complex FFT with the DC/Nyquist pair packed in
//              slot 0
//   axis 2   : forward complex FFT along k2
//   axis 1   : forward complex FFT along k1, fused with the K epilogue
//              q = K p and the p.q partial sums
//   postmix  : m = 0 plane, spectrum -> real parametrisation, K epilogue
// Each pencil FFT is a Stockham radix-R sequence: the first stage reads its
// inputs straight from global memory into registers, intermediate stages
// exchange through LDS, and the last stage writes from registers to global
// memory (or into the epilogue).  Strided passes map consecutive lanes to
// consecutive pencils, so every global access is a run of TM contiguous
// complex numbers.
#include "csipm_internal.h"

#include <cmath>
#include <type_traits>

namespace csipm {

namespace {

constexpr int kLdsBytes = 65536;     // LDS budget of an axis-3 workgroup

// ------------------------------------------------------------- radix plan --
template <int L, int E>
struct Radix {
  static constexpr int NT = L / E;
  static constexpr int nfull() {
    int c = 0, r = L;
    while (r >= E) { r /= E; ++c; }
    return c;
  }
  static constexpr int NFULL = nfull();
  static constexpr int rem() {
    int r = L;
    for (int i = 0; i < NFULL; ++i) r /= E;
    return r;
  }
  static constexpr int REM = rem();
  static constexpr int NSTAGES = NFULL + (REM > 1 ? 1 : 0);
  static constexpr int radix(int s) { return s < NFULL ? E : REM; }
  static constexpr int ns(int s) {
    int v = 1;
    for (int i = 0; i < s; ++i) v *= radix(i);
    return v;
  }
};

template <typename T, typename Tw>
__device__ __forceinline__ cx<T> twiddle(const Tw* tw, int idx, int dir) {
  cx<T> w = tw[idx];
  if (dir > 0) w.im = -w.im;
  return w;
}

// Applies stage S of a length-L Stockham FFT to the register block v (E
// values per thread: butterflies j = t + i*NT, i < E/r, value q at slot i*r+q).
template <typename T, int L, int E, int DIR, int S>
__device__ __forceinline__ void stage_compute(cx<T>* v, int t, const cx<T>* tw) {
  using RP = Radix<L, E>;
  constexpr int r = RP::radix(S);
  constexpr int Ns = RP::ns(S);
  constexpr int NT = RP::NT;
#pragma unroll
  for (int i = 0; i < E / r; ++i) {
    const int j = t + i * NT;
    if constexpr (Ns > 1) {
      const int jm = j % Ns;
#pragma unroll
      for (int q = 1; q < r; ++q) {
        v[i * r + q] = cmul(v[i * r + q], twiddle<T>(tw, jm * q * (L / (Ns * r)), DIR));
      }
    }
    dft_reg<r, DIR, T>(&v[i * r]);
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
  constexpr int r2 = RP::radix(S + 1);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < E / r; ++i) {
    const int j = t + i * NT;
    const int base = (j / Ns) * Ns * r + (j % Ns);
#pragma unroll
    for (int q = 0; q < r; ++q) lds[lidx(base + q * Ns)] = v[i * r + q];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < E / r2; ++i) {
    const int j = t + i * NT;
#pragma unroll
    for (int q = 0; q < r2; ++q) v[i * r2 + q] = lds[lidx(j + q * (L / r2))];
  }
}

// Runs all stages; inputs in the first-stage pattern, outputs left in
// registers in the last-stage pattern (element (t + i*NT) + q*(L/r_last)).
template <typename T, int L, int E, int DIR, int S, class LIdx>
__device__ __forceinline__ void fft_stages(cx<T>* v, int t, cx<T>* lds, LIdx lidx, const cx<T>* tw) {
  using RP = Radix<L, E>;
  stage_compute<T, L, E, DIR, S>(v, t, tw);
  if constexpr (S + 1 < RP::NSTAGES) {
    stage_exchange<T, L, E, S>(v, t, lds, lidx);
    fft_stages<T, L, E, DIR, S + 1>(v, t, lds, lidx, tw);
  }
}

template <typename T, int L, int E>
__device__ __forceinline__ int first_elem(int t, int i, int q) {
  using RP = Radix<L, E>;
  constexpr int r = RP::radix(0);
  return (t + i * RP::NT) + q * (L / r);
}
template <typename T, int L, int E>
__device__ __forceinline__ int last_elem(int t, int i, int q) {
  using RP = Radix<L, E>;
  constexpr int r = RP::radix(RP::NSTAGES - 1);
  return (t + i * RP::NT) + q * (L / r);
}
template <int L, int E, int S>
constexpr int radix_of() { return Radix<L, E>::radix(S); }

// ------------------------------------------------------- block reduction --
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block sums of NQ values; thread 0 writes out[q * stride + blockIdx.x].
// `red` is LDS scratch of at least NQ * NTHREADS/64 doubles; it may alias the
// FFT exchange buffer, so the block synchronises before writing it.
// The last NMAX quantities are maxima (of non-negative values), the others sums.
template <int NTHREADS, int NQ, int NMAX = 0>
__device__ __forceinline__ void block_sums_store(const double* v, double* out, int stride, double* red) {
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
// (m >= 1 there, the m = 0 plane in the postmix pass).
struct EpiNone {
  static constexpr int NRED = 0;
  static constexpr int NMAX = 0;
  double* partial = nullptr;
  int pstride = 0;
};

// q = K p (equation "condensedkkt" in Sigma form) and p.q
template <typename T>
struct EpiK {
  static constexpr int NRED = 1;
  static constexpr int NMAX = 0;
  KArgs<T> a;
  double* partial;
  int pstride;
  __device__ __forceinline__ void operator()(long long idx, cx<T> h, double* acc) const {
    const cx<T> pb = reinterpret_cast<const cx<T>*>(a.pb)[idx];
    const cx<T> pz = reinterpret_cast<const cx<T>*>(a.pz)[idx];
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
  RArgs a;
  double* partial;
  int pstride;
  __device__ __forceinline__ void operator()(long long idx, cx<double> h, double* acc) const {
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
// per workgroup TM (LDS = TM L w, at most 1024 threads).  Chosen from
// measurements at 256^3: 8 elements per thread for the FP64 axis-2 passes
// and the FP32 axis-1 forward pass, 16 otherwise; 128 KB tiles for axis 1
// except the FP64 inverse pass (64 KB), 64 KB for axis 2.
constexpr int strided_e(int w, int L, int axis, int dir) {
  const int e = ((w == 16 && axis == 2) || (w == 8 && axis == 1 && dir < 0)) ? 8 : 16;
  return L < e ? L : e;
}
constexpr int strided_lds(int w, int axis, int dir) {
  return axis == 2 ? 65536 : (w == 16 && dir > 0 ? 65536 : 131072);
}
constexpr int strided_tm(int w, int L, int axis, int dir) {
  int tm = strided_lds(w, axis, dir) / (L * w);
  if (tm > 64) tm = 64;
  if (tm < 1) tm = 1;
  while (tm * (L / strided_e(w, L, axis, dir)) > 1024) tm >>= 1;
  return tm;
}
template <typename T, int L, int AX, int DIR>
constexpr int strided_threads() {
  constexpr int w = int(sizeof(cx<T>));
  return strided_tm(w, L, AX, DIR) * (L / strided_e(w, L, AX, DIR));
}

template <typename T, int L, int AX, int DIR, class Epi>
__global__ void __launch_bounds__((strided_threads<T, L, AX, DIR>()))
k_axis12(const cx<T>* src, cx<T>* dst, StridedGeom<T> geo,
         const cx<T>* __restrict__ tw, int m, int m0_from_dst, Epi epi, const int* skip) {
  if (skip && *skip) return;
  constexpr int E = strided_e(int(sizeof(cx<T>)), L, AX, DIR);
  constexpr int TM = strided_tm(int(sizeof(cx<T>)), L, AX, DIR);
  constexpr int NT = L / E;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int p = threadIdx.x % TM;
  const int t = threadIdx.x / TM;
  const int qpen = blockIdx.x * TM + p;
  const bool active = qpen < geo.batch;
  const long long base = active ? (long long)(qpen / geo.inner) * geo.outer + (qpen % geo.inner) : 0;
  const bool is_m0 = (qpen % m) == 0;
  const cx<T>* in = (m0_from_dst && is_m0) ? dst : src;

  cx<T> v[E];
  constexpr int r0 = radix_of<L, E, 0>();
#pragma unroll
  for (int i = 0; i < E / r0; ++i)
#pragma unroll
    for (int q = 0; q < r0; ++q) {
      const int e = first_elem<T, L, E>(t, i, q);
      v[i * r0 + q] = active ? in[base + (long long)e * geo.estride] : cx<T>{T(0), T(0)};
    }
  auto lidx = [p](int e) { return e * TM + p; };
  fft_stages<T, L, E, DIR, 0>(v, t, lds, lidx, tw);

  constexpr int rl = radix_of<L, E, Radix<L, E>::NSTAGES - 1>();
  if constexpr (Epi::NRED > 0) {
    double acc[Epi::NRED];
#pragma unroll
    for (int q = 0; q < Epi::NRED; ++q) acc[q] = 0.0;
    if (active) {
#pragma unroll
      for (int i = 0; i < E / rl; ++i)
#pragma unroll
        for (int q = 0; q < rl; ++q) {
          const long long idx = base + (long long)last_elem<T, L, E>(t, i, q) * geo.estride;
          if (is_m0)
            dst[idx] = v[i * rl + q];   // finished by the postmix pass
          else
            epi(idx, v[i * rl + q], acc);
        }
    }
    block_sums_store<TM * NT, Epi::NRED, Epi::NMAX>(acc, epi.partial, epi.pstride,
                                                    reinterpret_cast<double*>(smem_raw));
  } else {
    if (active) {
#pragma unroll
      for (int i = 0; i < E / rl; ++i)
#pragma unroll
        for (int q = 0; q < rl; ++q) {
          const int e = last_elem<T, L, E>(t, i, q);
          dst[base + (long long)e * geo.estride] = v[i * rl + q];
        }
    }
  }
}

// ------------------------------------------------------ axis-3 (c2r/r2c) --
template <typename T>
constexpr int a3_e(int L) { return L < 8 ? L : 8; }   // 8 elements per thread (measured best)
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
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* ldsall = reinterpret_cast<cx<T>*>(smem_raw);
  const int p = threadIdx.x / NT;
  const int t = threadIdx.x % NT;
  const int pen = blockIdx.x * PP + p;
  const bool active = pen < npencils;
  const long long base = (long long)pen * L;
  cx<T>* lds = ldsall + p * LP;
  auto lidx = [](int e) { return e + (e >> 4); };
  const T rs2 = T(0.70710678118654752440);

  cx<T> v[E];
  if constexpr (MODE & A3_C2R) {
    // stage the packed half-spectrum through LDS: Z_e needs X_e and X_{L-e}
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int e = t + q * NT;
      lds[lidx(e)] = active ? src[base + e] : cx<T>{T(0), T(0)};
    }
    __syncthreads();
    constexpr int r0 = radix_of<L, E, 0>();
#pragma unroll
    for (int i = 0; i < E / r0; ++i)
#pragma unroll
      for (int q = 0; q < r0; ++q) {
        const int e = first_elem<T, L, E>(t, i, q);
        cx<T> z;
        if (e == 0) {
          const cx<T> x0 = lds[lidx(0)];   // (DC, Nyquist)
          z = {x0.re + x0.im, x0.re - x0.im};
        } else {
          const cx<T> a = cscale(lds[lidx(e)], rs2);
          const cx<T> b = cconj(cscale(lds[lidx(L - e)], rs2));
          const cx<T> s = cadd(a, b);
          const cx<T> d = csub(a, b);
          cx<T> w = tw3[e];          // exp(-2 pi i e / N3)
          w.im = -w.im;              // exp(+2 pi i e / N3)
          const cx<T> id = cmul_i<1>(cmul(w, d));
          z = cadd(s, id);
        }
        v[i * r0 + q] = z;
      }
    fft_stages<T, L, E, +1, 0>(v, t, lds, lidx, twm);
    constexpr int rl = radix_of<L, E, Radix<L, E>::NSTAGES - 1>();
    // z_e = x[2e] + i x[2e+1]
#pragma unroll
    for (int i = 0; i < E / rl; ++i)
#pragma unroll
      for (int q = 0; q < rl; ++q) {
        const int e = last_elem<T, L, E>(t, i, q);
        cx<T> z = cscale(v[i * rl + q], sc_c2r);
        if constexpr (MODE == A3_FULL) {
          const long long bit = (long long)pen * N3 + 2 * e;
          const uint32_t wd = active ? mask[bit >> 5] : 0u;
          const int sh = (int)(bit & 31);
          if (!((wd >> sh) & 1u)) z.re = T(0);
          if (!((wd >> (sh + 1)) & 1u)) z.im = T(0);
        }
        v[i * rl + q] = z;
      }
    if constexpr (MODE == A3_C2R) {
      if (active) {
#pragma unroll
        for (int i = 0; i < E / rl; ++i)
#pragma unroll
          for (int q = 0; q < rl; ++q) dst[base + last_elem<T, L, E>(t, i, q)] = v[i * rl + q];
      }
      return;
    } else {
      // re-order to the first-stage pattern of the forward transform
      __syncthreads();
#pragma unroll
      for (int i = 0; i < E / rl; ++i)
#pragma unroll
        for (int q = 0; q < rl; ++q) lds[lidx(last_elem<T, L, E>(t, i, q))] = v[i * rl + q];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < E / r0; ++i)
#pragma unroll
        for (int q = 0; q < r0; ++q) v[i * r0 + q] = lds[lidx(first_elem<T, L, E>(t, i, q))];
    }
  } else {
    constexpr int r0 = radix_of<L, E, 0>();
#pragma unroll
    for (int i = 0; i < E / r0; ++i)
#pragma unroll
      for (int q = 0; q < r0; ++q) {
        const int e = first_elem<T, L, E>(t, i, q);
        v[i * r0 + q] = active ? src[base + e] : cx<T>{T(0), T(0)};
      }
  }

  // forward half-length FFT of z' and the r2c post-processing
  fft_stages<T, L, E, -1, 0>(v, t, lds, lidx, twm);
  constexpr int rl = radix_of<L, E, Radix<L, E>::NSTAGES - 1>();
  __syncthreads();
#pragma unroll
  for (int i = 0; i < E / rl; ++i)
#pragma unroll
    for (int q = 0; q < rl; ++q) lds[lidx(last_elem<T, L, E>(t, i, q))] = v[i * rl + q];
  __syncthreads();
  if (!active) return;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int e = t + q * NT;
    cx<T> xo;
    if (e == 0) {
      const cx<T> z0 = lds[lidx(0)];
      xo = {(z0.re + z0.im) * sc_r2c_dc, (z0.re - z0.im) * sc_r2c_dc};
    } else {
      const cx<T> a = lds[lidx(e)];
      const cx<T> b = cconj(lds[lidx(L - e)]);
      const cx<T> ev = cscale(cadd(a, b), T(0.5));
      const cx<T> od = cscale(csub(a, b), T(0.5));
      const cx<T> w = tw3[e];        // exp(-2 pi i e / N3)
      const cx<T> t2 = cmul_i<-1>(cmul(w, od));
      xo = cscale(cadd(ev, t2), sc_r2c);
    }
    dst[base + e] = xo;
  }
}

// --------------------------------------------------------- m = 0 mixing --
// 2D class of (k1, k2) in the m = 0 plane: 0 self-conjugate, 1 canonical,
// 2 mirror of a canonical index.
__device__ __forceinline__ int cls2(int k1, int k2, int n1, int n2) {
  const bool e1 = (2 * k1 == n1) || k1 == 0;
  const bool e2 = (2 * k2 == n2) || k2 == 0;
  if (e1 && e2) return 0;
  if (2 * k2 < n2 && k2 >= 1) return 1;
  if (e2 && k1 >= 1 && 2 * k1 < n1) return 1;
  return 2;
}

template <typename T>
__global__ void k_premix(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, int n1, int n2, int m,
                         const int* skip) {
  if (skip && *skip) return;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n1 * n2) return;
  const int k1 = id / n2, k2 = id % n2;
  const int c = cls2(k1, k2, n1, n2);
  if (c == 2) return;
  const long long ia = ((long long)k1 * n2 + k2) * m;
  if (c == 0) {
    dst[ia] = src[ia];
    return;
  }
  const int q1 = (n1 - k1) % n1, q2 = (n2 - k2) % n2;
  const long long ib = ((long long)q1 * n2 + q2) * m;
  const T r = T(0.70710678118654752440);
  const cx<T> a = src[ia], b = src[ib];
  // U[k] = (W[k] + i W[-k]) / sqrt2,  U[-k] = (W[k] - i W[-k]) / sqrt2
  const cx<T> ib_ = cmul_i<1>(b);
  dst[ia] = cscale(cadd(a, ib_), r);
  dst[ib] = cscale(csub(a, ib_), r);
}

template <typename T, class Epi>
__global__ void __launch_bounds__(256)
k_postmix(const cx<T>* work, cx<T>* out, int n1, int n2, int m, Epi epi, const int* skip) {
  if (skip && *skip) return;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  double acc[Epi::NRED > 0 ? Epi::NRED : 1];
#pragma unroll
  for (int q = 0; q < (Epi::NRED > 0 ? Epi::NRED : 1); ++q) acc[q] = 0.0;
  if (id < n1 * n2) {
    const int k1 = id / n2, k2 = id % n2;
    const int c = cls2(k1, k2, n1, n2);
    if (c != 2) {
      const long long ia = ((long long)k1 * n2 + k2) * m;
      const int q1 = (n1 - k1) % n1, q2 = (n2 - k2) % n2;
      const long long ib = ((long long)q1 * n2 + q2) * m;
      cx<T> ha, hb;
      int cnt;
      if (c == 0) {
        ha = work[ia];
        cnt = 1;
      } else {
        const T r = T(0.70710678118654752440);
        const cx<T> a = work[ia], b = work[ib];
        // W[k] = (U[k] + U[-k]) / sqrt2,  W[-k] = i (U[-k] - U[k]) / sqrt2
        ha = cscale(cadd(a, b), r);
        hb = cscale(cmul_i<1>(csub(b, a)), r);
        cnt = 2;
      }
      if constexpr (Epi::NRED > 0) {
        epi(ia, ha, acc);
        if (cnt == 2) epi(ib, hb, acc);
      } else {
        out[ia] = ha;
        if (cnt == 2) out[ib] = hb;
      }
    }
  }
  if constexpr (Epi::NRED > 0) {
    __shared__ double red[4 * Epi::NRED];
    block_sums_store<256, Epi::NRED, Epi::NMAX>(acc, epi.partial, epi.pstride, red);
  }
}

// ----------------------------------------------------- layout conversion --
// internal real index r = ((k1*N2 + k2)*M + m)*2 + part
__device__ __forceinline__ long long ext_index(long long r, int n1, int n2, int n3, int m) {
  const int part = (int)(r & 1);
  const long long c = r >> 1;
  const int mm = (int)(c % m);
  const long long c2 = c / m;
  const int k2 = (int)(c2 % n2);
  const int k1 = (int)(c2 / n2);
  int e1 = k1, e2 = k2, e3;
  if (mm == 0) {
    e3 = part ? m : 0;
  } else if (part == 0) {
    e3 = mm;
  } else {
    e1 = (n1 - k1) % n1;
    e2 = (n2 - k2) % n2;
    e3 = n3 - mm;
  }
  return ((long long)e1 * n2 + e2) * n3 + e3;
}

template <typename Te, typename Ti>
__global__ void k_to_internal(const Te* __restrict__ ext, Ti* __restrict__ in, long long n, int n1,
                              int n2, int n3, int m) {
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < n;
       r += (long long)gridDim.x * blockDim.x)
    in[r] = (Ti)ext[ext_index(r, n1, n2, n3, m)];
}

template <typename Ti, typename Te>
__global__ void k_to_external(const Ti* __restrict__ in, Te* __restrict__ ext, long long n, int n1,
                              int n2, int n3, int m) {
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < n;
       r += (long long)gridDim.x * blockDim.x)
    ext[ext_index(r, n1, n2, n3, m)] = (Te)in[r];
}

__global__ void k_feat_to_external(const float4* __restrict__ in, float4* __restrict__ ext, long long n, int n1,
                                   int n2, int n3, int m) {
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < n;
       r += (long long)gridDim.x * blockDim.x)
    ext[ext_index(r, n1, n2, n3, m)] = in[r];
}

__global__ void k_pack_mask(const uint8_t* __restrict__ obs, uint32_t* __restrict__ bits, long long nwords) {
  for (long long w = blockIdx.x * (long long)blockDim.x + threadIdx.x; w < nwords;
       w += (long long)gridDim.x * blockDim.x) {
    uint32_t v = 0;
    for (int b = 0; b < 32; ++b) v |= (obs[w * 32 + b] ? 1u : 0u) << b;
    bits[w] = v;
  }
}

int grid_for(long long n, int block) {
  long long g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename T, int AX, int DIR, class Epi>
void launch_axis12_L(int L, dim3 grid, const cx<T>* src, cx<T>* dst, StridedGeom<T> geo, const cx<T>* tw,
                     int m, int m0, Epi epi, const int* skip, hipStream_t s) {
#define CSIPM_A12(LL)                                                                               \
  case LL: {                                                                                        \
    constexpr int TM = strided_tm(int(sizeof(cx<T>)), LL, AX, DIR);                                \
    constexpr int NT = LL / strided_e(int(sizeof(cx<T>)), LL, AX, DIR);                             \
    const size_t shm = (size_t)TM * LL * sizeof(cx<T>);                                             \
    auto kern = k_axis12<T, LL, AX, DIR, Epi>;                                                      \
    if (shm > 65536) (void)hipFuncSetAttribute((const void*)kern,                                   \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm); \
    hipLaunchKernelGGL(kern, grid, dim3(TM * NT), shm, s, src, dst, geo, tw, m, m0, epi, skip);      \
    break;                                                                                          \
  }
  switch (L) {
    CSIPM_A12(4)
    CSIPM_A12(8)
    CSIPM_A12(16)
    CSIPM_A12(32)
    CSIPM_A12(64)
    CSIPM_A12(128)
    CSIPM_A12(256)
    CSIPM_A12(512)
    CSIPM_A12(1024)
    default:
      break;
  }
#undef CSIPM_A12
}

template <typename T>
StridedGeom<T> geom(const Grid& g, int axis) {
  StridedGeom<T> geo;
  if (axis == 1) {
    geo.inner = g.n2 * g.m;
    geo.outer = 0;
    geo.estride = (long long)g.n2 * g.m;
    geo.batch = g.n2 * g.m;
  } else {
    geo.inner = g.m;
    geo.outer = (long long)g.n2 * g.m;
    geo.estride = g.m;
    geo.batch = g.n1 * g.m;
  }
  return geo;
}

}  // namespace

int axis12_blocks(const Grid& g, int axis, int elem_bytes, int dir) {
  const int L = axis == 1 ? g.n1 : g.n2;
  const int batch = axis == 1 ? g.n2 * g.m : g.n1 * g.m;
  const int tm = strided_tm(elem_bytes, L, axis, dir);
  return (batch + tm - 1) / tm;
}

int postmix_blocks(const Grid& g) { return (g.n1 * g.n2 + 255) / 256; }

template <typename T>
void launch_premix(const Grid& g, const T* src, T* work, const int* skip, hipStream_t s) {
  const int tot = g.n1 * g.n2;
  hipLaunchKernelGGL((k_premix<T>), dim3((tot + 255) / 256), dim3(256), 0, s,
                     reinterpret_cast<const cx<T>*>(src), reinterpret_cast<cx<T>*>(work), g.n1, g.n2, g.m, skip);
}

template <typename T>
void launch_axis12(const Grid& g, int axis, int dir, const T* src, T* dst, const Twiddles<T>& tw, int epi,
                   const EpiArgs<T>* ea, bool m0_from_dst, const int* skip, hipStream_t s) {
  const int L = axis == 1 ? g.n1 : g.n2;
  const cx<T>* twp = axis == 1 ? tw.t1 : tw.t2;
  StridedGeom<T> geo = geom<T>(g, axis);
  dim3 grid(axis12_blocks(g, axis, (int)sizeof(cx<T>), dir));
  const cx<T>* cs = reinterpret_cast<const cx<T>*>(src);
  cx<T>* cd = reinterpret_cast<cx<T>*>(dst);
  if (axis == 1) {
    if (dir > 0) {
      launch_axis12_L<T, 1, +1>(L, grid, cs, cd, geo, twp, g.m, m0_from_dst ? 1 : 0, EpiNone{}, skip, s);
    } else if (epi == EPI_K) {
      launch_axis12_L<T, 1, -1>(L, grid, cs, cd, geo, twp, g.m, 0, EpiK<T>{ea->k, ea->partial, ea->pstride}, skip, s);
    } else if (epi == EPI_R) {
      if constexpr (std::is_same<T, double>::value)
        launch_axis12_L<T, 1, -1>(L, grid, cs, cd, geo, twp, g.m, 0, EpiR{ea->r, ea->partial, ea->pstride}, skip, s);
    } else {
      launch_axis12_L<T, 1, -1>(L, grid, cs, cd, geo, twp, g.m, 0, EpiNone{}, skip, s);
    }
  } else {
    if (dir > 0)
      launch_axis12_L<T, 2, +1>(L, grid, cs, cd, geo, twp, g.m, 0, EpiNone{}, skip, s);
    else
      launch_axis12_L<T, 2, -1>(L, grid, cs, cd, geo, twp, g.m, 0, EpiNone{}, skip, s);
  }
}

template <typename T>
void launch_axis3(const Grid& g, int mode, const T* src, T* dst, const uint32_t* maskbits, const Twiddles<T>& tw,
                  const int* skip, hipStream_t s) {
  const int L = g.m;
  const int np = g.n1 * g.n2;
  const double rn = 1.0 / std::sqrt((double)g.n);
  const T sc_c2r = (T)rn;
  const T sc_dc = (T)rn;
  const T sc_ac = (T)(rn * std::sqrt(2.0));
  const cx<T>* cs = reinterpret_cast<const cx<T>*>(src);
  cx<T>* cd = reinterpret_cast<cx<T>*>(dst);
#define CSIPM_A3(LL)                                                                               \
  case LL: {                                                                                       \
    constexpr int PP = a3_pp<T>(LL);                                                               \
    constexpr int NT = LL / a3_e<T>(LL);                                                           \
    const size_t shm = (size_t)PP * a3_pad<T>(LL) * sizeof(cx<T>);                                 \
    dim3 grid((np + PP - 1) / PP), block(PP * NT);                                                 \
    if (shm > 65536) {                                                                             \
      (void)hipFuncSetAttribute((const void*)k_axis3<T, LL, A3_FULL>,                              \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);            \
      (void)hipFuncSetAttribute((const void*)k_axis3<T, LL, A3_C2R>,                               \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);            \
      (void)hipFuncSetAttribute((const void*)k_axis3<T, LL, A3_R2C>,                               \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);            \
    }                                                                                              \
    if (mode == A3_FULL)                                                                           \
      hipLaunchKernelGGL((k_axis3<T, LL, A3_FULL>), grid, block, shm, s, cs, cd, maskbits, tw.tm, \
                         tw.t3, np, sc_c2r, sc_dc, sc_ac, skip);                                         \
    else if (mode == A3_C2R)                                                                       \
      hipLaunchKernelGGL((k_axis3<T, LL, A3_C2R>), grid, block, shm, s, cs, cd, maskbits, tw.tm,  \
                         tw.t3, np, sc_c2r, sc_dc, sc_ac, skip);                                         \
    else                                                                                           \
      hipLaunchKernelGGL((k_axis3<T, LL, A3_R2C>), grid, block, shm, s, cs, cd, maskbits, tw.tm,  \
                         tw.t3, np, sc_c2r, sc_dc, sc_ac, skip);                                         \
    break;                                                                                         \
  }
  switch (L) {
    CSIPM_A3(2)
    CSIPM_A3(4)
    CSIPM_A3(8)
    CSIPM_A3(16)
    CSIPM_A3(32)
    CSIPM_A3(64)
    CSIPM_A3(128)
    CSIPM_A3(256)
    CSIPM_A3(512)
    default:
      break;
  }
#undef CSIPM_A3
}

template <typename T>
void launch_postmix(const Grid& g, const T* work, T* out, int epi, const EpiArgs<T>* ea, const int* skip,
                    hipStream_t s) {
  dim3 grid(postmix_blocks(g));
  const cx<T>* w = reinterpret_cast<const cx<T>*>(work);
  cx<T>* o = reinterpret_cast<cx<T>*>(out);
  if (epi == EPI_K) {
    hipLaunchKernelGGL((k_postmix<T, EpiK<T>>), grid, dim3(256), 0, s, w, o, g.n1, g.n2, g.m,
                       EpiK<T>{ea->k, ea->partial, ea->pstride}, skip);
  } else if (epi == EPI_R) {
    if constexpr (std::is_same<T, double>::value)
      hipLaunchKernelGGL((k_postmix<T, EpiR>), grid, dim3(256), 0, s, w, o, g.n1, g.n2, g.m,
                         EpiR{ea->r, ea->partial, ea->pstride}, skip);
  } else {
    hipLaunchKernelGGL((k_postmix<T, EpiNone>), grid, dim3(256), 0, s, w, o, g.n1, g.n2, g.m, EpiNone{}, skip);
  }
}

template <typename Te, typename Ti>
void launch_to_internal(const Grid& g, const Te* ext, Ti* in, hipStream_t s) {
  hipLaunchKernelGGL((k_to_internal<Te, Ti>), dim3(grid_for(g.n, 256)), dim3(256), 0, s, ext, in, g.n, g.n1,
                     g.n2, g.n3, g.m);
}
template <typename Ti, typename Te>
void launch_to_external(const Grid& g, const Ti* in, Te* ext, hipStream_t s) {
  hipLaunchKernelGGL((k_to_external<Ti, Te>), dim3(grid_for(g.n, 256)), dim3(256), 0, s, in, ext, g.n, g.n1,
                     g.n2, g.n3, g.m);
}
void launch_feat_to_external(const Grid& g, const float* in, float* ext, hipStream_t s) {
  hipLaunchKernelGGL(k_feat_to_external, dim3(grid_for(g.n, 256)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(in), reinterpret_cast<float4*>(ext), g.n, g.n1, g.n2, g.n3,
                     g.m);
}
void launch_pack_mask(const Grid& g, const uint8_t* obs, uint32_t* bits, hipStream_t s) {
  const long long nw = g.n / 32;
  hipLaunchKernelGGL(k_pack_mask, dim3(grid_for(nw, 256)), dim3(256), 0, s, obs, bits, nw);
}

#define CSIPM_INST(T)                                                                                          \
  template void launch_premix<T>(const Grid&, const T*, T*, const int*, hipStream_t);                          \
  template void launch_axis12<T>(const Grid&, int, int, const T*, T*, const Twiddles<T>&, int,                 \
                                 const EpiArgs<T>*, bool, const int*, hipStream_t);                            \
  template void launch_axis3<T>(const Grid&, int, const T*, T*, const uint32_t*, const Twiddles<T>&,           \
                                const int*, hipStream_t);                                                      \
  template void launch_postmix<T>(const Grid&, const T*, T*, int, const EpiArgs<T>*, const int*, hipStream_t); \
  template void launch_to_internal<double, T>(const Grid&, const double*, T*, hipStream_t);                   \
  template void launch_to_internal<float, T>(const Grid&, const float*, T*, hipStream_t);                     \
  template void launch_to_external<T, double>(const Grid&, const T*, double*, hipStream_t);                   \
  template void launch_to_external<T, float>(const Grid&, const T*, float*, hipStream_t);
CSIPM_INST(double)
CSIPM_INST(float)
#undef CSIPM_INST

}  // namespace csipm
