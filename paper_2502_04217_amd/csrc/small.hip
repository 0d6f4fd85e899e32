// Batches of small problems solved in one launch: one workgroup runs the
// whole interior-point solve of one problem (paper: sec. "Primal-dual
// interior-point method", equations "kkt", "kktmu" and "condensedkkt"; the
// Newton systems by PCG with the paper's preconditioner, equation
// "invprecond1"), with every scalar decision taken on the device, so a
// batch needs no host round trip until it is done.
//
// The steps are those of the library's standard form in FP64 (the readings
// of the barrier strategy, right-hand side and stopping rules), on the
// simplest data path: H beta is recomputed by a full H-apply at every
// iterate, and the operators run on the whole Hermitian spectrum, one axis
// at a time, in place: a pencil of power-of-two length up to 32 is
// transformed by one thread in registers (radix 2), any other length up to
// kSmallMaxExtent by direct DFTs (L^2 work per pencil) through a second
// buffer.  The spectrum sits in LDS when it fits (kSmallLdsBytes), else in
// the problem's workspace.  A problem's result does not depend on the
// others in the batch: a batch of one gives the same bits.
#include "small.h"

#include "../../include/csipm.h"

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

namespace csipm {

namespace {

constexpr int kSmallThreads = 512;
constexpr int kSmallWaves = kSmallThreads / 64;

struct SmallDims {
  int n1, n2, n3;
  long long n;
};

// ------------------------------------------------------- block reductions --
// (every thread of the workgroup calls these; red holds kSmallWaves doubles)
// op 0: sum, 1: max, 2: min; the waves' values combined in wave order
__device__ double block_reduce(double v, int op, double* red) {
  v = op == 0 ? wave_sum(v) : op == 1 ? wave_max(v) : wave_min(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double a = red[0];
  for (int k = 1; k < kSmallWaves; ++k) a = op == 0 ? a + red[k] : op == 1 ? fmax(a, red[k]) : fmin(a, red[k]);
  return a;
}

// ------------------------------------------------------------- transforms --
__device__ __forceinline__ void unravel(long long f, const SmallDims& d, int& k1, int& k2, int& k3) {
  k3 = (int)(f % d.n3);
  const long long r = f / d.n3;
  k2 = (int)(r % d.n2);
  k1 = (int)(r / d.n2);
}
__device__ __forceinline__ long long mirror_of(int k1, int k2, int k3, const SmallDims& d) {
  const int m1 = k1 ? d.n1 - k1 : 0, m2 = k2 ? d.n2 - k2 : 0, m3 = k3 ? d.n3 - k3 : 0;
  return ((long long)m1 * d.n2 + m2) * d.n3 + m3;
}

// One direct DFT pass along `axis` (1, 2, 3) from src to dst: dst[.., k, ..]
// = sum_j src[.., j, ..] exp(dir 2 pi i j k / L), the sum taken in order j =
// 0, 1, ..., L - 1 with tw[q] = exp(-2 pi i q / L) from the host tables.
__device__ void dft_pass(const cx<double>* src, cx<double>* dst, const SmallDims& d, int axis, int dir,
                         const cx<double>* tw) {
  const int L = axis == 1 ? d.n1 : axis == 2 ? d.n2 : d.n3;
  const long long st = axis == 1 ? (long long)d.n2 * d.n3 : axis == 2 ? d.n3 : 1;
  for (long long f = threadIdx.x; f < d.n; f += kSmallThreads) {
    int k1, k2, k3;
    unravel(f, d, k1, k2, k3);
    const int k = axis == 1 ? k1 : axis == 2 ? k2 : k3;
    const long long base = f - (long long)k * st;
    double re = 0.0, im = 0.0;
    int q = 0;   // j k mod L
    for (int j = 0; j < L; ++j) {
      const cx<double> x = src[base + (long long)j * st];
      const cx<double> w = tw[q];
      const double wi = dir > 0 ? -w.im : w.im;
      re += x.re * w.re - x.im * wi;
      im += x.re * wi + x.im * w.re;
      q += k;
      if (q >= L) q -= L;
    }
    dst[f] = {re, im};
  }
  __syncthreads();
}

constexpr int bitrev(int j, int L) {
  int r = 0;
  for (int b = 1; b < L; b <<= 1) {
    r = (r << 1) | (j & 1);
    j >>= 1;
  }
  return r;
}

// pencils of length L (a power of two) transformed in place, one per
// thread: loaded in bit-reversed order, radix-2 butterflies in registers
// (span len, twiddles tw[k L / len]), written back in order
template <int L>
__device__ void reg_pass(cx<double>* w, const SmallDims& d, int axis, int dir, const cx<double>* tw) {
  const long long st = axis == 1 ? (long long)d.n2 * d.n3 : axis == 2 ? d.n3 : 1;
  const long long npen = d.n / L;
  for (long long P = threadIdx.x; P < npen; P += kSmallThreads) {
    const long long base =
        axis == 1 ? P : axis == 2 ? (P / d.n3) * ((long long)d.n2 * d.n3) + P % d.n3 : P * (long long)d.n3;
    cx<double> v[L];
#pragma unroll
    for (int j = 0; j < L; ++j) v[bitrev(j, L)] = w[base + (long long)j * st];
#pragma unroll
    for (int len = 2; len <= L; len <<= 1) {
      const int half = len >> 1, step = L / len;
#pragma unroll
      for (int i = 0; i < L; i += len)
#pragma unroll
        for (int k = 0; k < half; ++k) {
          const cx<double> t0 = tw[k * step];
          const double wr = t0.re, wi = dir > 0 ? -t0.im : t0.im;
          const cx<double> a = v[i + k], b = v[i + k + half];
          const double tr = b.re * wr - b.im * wi, ti = b.re * wi + b.im * wr;
          v[i + k] = {a.re + tr, a.im + ti};
          v[i + k + half] = {a.re - tr, a.im - ti};
        }
    }
#pragma unroll
    for (int j = 0; j < L; ++j) w[base + (long long)j * st] = v[j];
  }
  __syncthreads();
}

// whether an extent takes the register pass (else the direct DFT)
__host__ __device__ constexpr bool reg_length(int L) { return L == 2 || L == 4 || L == 8 || L == 16 || L == 32; }

// one axis of the full-spectrum transform of w, in place (scr: n complex of
// scratch for the direct DFT of other lengths).  RMAX is the longest
// register pencil the kernel instance holds (32 takes about twice the
// registers of 16, so grids without a 32-point axis use the 16 instance).
template <int RMAX>
__device__ void axis_pass(cx<double>* w, cx<double>* scr, const SmallDims& d, int axis, int dir,
                          const cx<double>* tw) {
  const int L = axis == 1 ? d.n1 : axis == 2 ? d.n2 : d.n3;
  if constexpr (RMAX >= 32) {
    if (L == 32) {
      reg_pass<32>(w, d, axis, dir, tw);
      return;
    }
  }
  switch (L) {
    case 1:
      return;
    case 2:
      reg_pass<2>(w, d, axis, dir, tw);
      return;
    case 4:
      reg_pass<4>(w, d, axis, dir, tw);
      return;
    case 8:
      reg_pass<8>(w, d, axis, dir, tw);
      return;
    case 16:
      reg_pass<16>(w, d, axis, dir, tw);
      return;
    default:
      dft_pass(w, scr, d, axis, dir, tw);
      for (long long f = threadIdx.x; f < d.n; f += kSmallThreads) w[f] = scr[f];
      __syncthreads();
      return;
  }
}

struct SmallTw {
  const cx<double>* t1;
  const cx<double>* t2;
  const cx<double>* t3;
};

// y = H beta = A^T D A beta (beta and y in the external parametrisation of
// derivation "map"); w0 holds the n-point spectrum, scr n complex of scratch.
template <int RMAX>
__device__ void h_apply(const double* beta, double* y, const uint8_t* obs, const SmallDims& d, const SmallTw& tw,
                        cx<double>* w0, cx<double>* scr) {
  const double rs2 = 0.70710678118654752440, sq2 = 1.41421356237309504880;
  for (long long f = threadIdx.x; f < d.n; f += kSmallThreads) {
    int k1, k2, k3;
    unravel(f, d, k1, k2, k3);
    const int c = cls3(k1, k2, k3, d.n1, d.n2, d.n3);
    const double b = beta[f];
    if (c == 0) {
      w0[f] = {b, 0.0};
    } else {
      const double bm = beta[mirror_of(k1, k2, k3, d)];
      w0[f] = c == 1 ? cx<double>{rs2 * b, rs2 * bm} : cx<double>{rs2 * bm, -rs2 * b};
    }
  }
  __syncthreads();
  axis_pass<RMAX>(w0, scr, d, 1, +1, tw.t1);
  axis_pass<RMAX>(w0, scr, d, 2, +1, tw.t2);
  axis_pass<RMAX>(w0, scr, d, 3, +1, tw.t3);
  const double sc = 1.0 / (double)d.n;   // both unitary normalisations
  for (long long f = threadIdx.x; f < d.n; f += kSmallThreads) w0[f] = {obs[f] ? w0[f].re * sc : 0.0, 0.0};
  __syncthreads();
  axis_pass<RMAX>(w0, scr, d, 3, -1, tw.t3);
  axis_pass<RMAX>(w0, scr, d, 2, -1, tw.t2);
  axis_pass<RMAX>(w0, scr, d, 1, -1, tw.t1);
  for (long long f = threadIdx.x; f < d.n; f += kSmallThreads) {
    int k1, k2, k3;
    unravel(f, d, k1, k2, k3);
    const int c = cls3(k1, k2, k3, d.n1, d.n2, d.n3);
    const cx<double> h = w0[f];
    y[f] = c == 0 ? h.re : (c == 1 ? sq2 * h.re : -sq2 * h.im);
  }
  __syncthreads();
}

// xi = A^T b_hat = B DFT(b_hat) (the adjoint of A, reading "adjoint")
template <int RMAX>
__device__ void at_apply(const double* x, const uint8_t* obs, double* out, const SmallDims& d, const SmallTw& tw,
                         cx<double>* w0, cx<double>* scr) {
  const double sq2 = 1.41421356237309504880;
  const double sc = 1.0 / sqrt((double)d.n);
  for (long long f = threadIdx.x; f < d.n; f += kSmallThreads) w0[f] = {obs[f] ? x[f] * sc : 0.0, 0.0};
  __syncthreads();
  axis_pass<RMAX>(w0, scr, d, 3, -1, tw.t3);
  axis_pass<RMAX>(w0, scr, d, 2, -1, tw.t2);
  axis_pass<RMAX>(w0, scr, d, 1, -1, tw.t1);
  for (long long f = threadIdx.x; f < d.n; f += kSmallThreads) {
    int k1, k2, k3;
    unravel(f, d, k1, k2, k3);
    const int c = cls3(k1, k2, k3, d.n1, d.n2, d.n3);
    const cx<double> h = w0[f];
    out[f] = c == 0 ? h.re : (c == 1 ? sq2 * h.re : -sq2 * h.im);
  }
  __syncthreads();
}

// P^{-1} of one 2x2 block (equation "invprecond1", C = I)
__device__ __forceinline__ void pinv1(double rb, double rz, double s1, double s2, double& zb, double& zz) {
  const double L1 = s1 + s2, L2 = s1 - s2;
  const double D = L1 + 4.0 * s1 * s2;
  zb = (L1 * rb - L2 * rz) / D;
  zz = (-L2 * rb + (1.0 + L1) * rz) / D;
}

// largest a with v + a dv >= 0 over this thread's share (inf if none)
__device__ __forceinline__ double ratio(double v, double dv) { return dv < 0.0 ? -v / dv : INFINITY; }

// the per-problem arrays, each of n doubles, in the problem's workspace
enum SmallVec {
  SV_XI, SV_B, SV_Z, SV_N1, SV_N2, SV_HB, SV_S1, SV_S2, SV_XB, SV_XZ, SV_RB, SV_RZ, SV_PB, SV_PZ, SV_QB, SV_QZ,
  SV_COUNT
};

template <int RMAX>
__global__ void __launch_bounds__(kSmallThreads)
k_small_solve(int n1, int n2, int n3, const double* __restrict__ signals, const uint8_t* __restrict__ observed,
              const double* __restrict__ lambdas, double lambda_frac, double* __restrict__ beta_out,
              double* __restrict__ info, char* __restrict__ ws, long long ws_stride, const cx<double>* __restrict__ tw,
              SmallOpts o, int lds_spectrum) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[kSmallWaves];
  const SmallDims d{n1, n2, n3, (long long)n1 * n2 * n3};
  const long long n = d.n;
  const int p = blockIdx.x;
  const double* sig = signals + (long long)p * n;
  const uint8_t* obs = observed + (long long)p * n;
  double* v = reinterpret_cast<double*>(ws + (long long)p * ws_stride);
  // the spectrum and, for a length without the register pass, its scratch
  cx<double>* w0 = lds_spectrum ? reinterpret_cast<cx<double>*>(smem)
                                : reinterpret_cast<cx<double>*>(v + (long long)SV_COUNT * n);
  cx<double>* w1 = w0 + n;
  const SmallTw T{tw, tw + n1, tw + n1 + n2};
  double *xi = v + SV_XI * n, *be = v + SV_B * n, *zv = v + SV_Z * n, *nu1 = v + SV_N1 * n,
         *nu2 = v + SV_N2 * n, *hb = v + SV_HB * n, *g1 = v + SV_S1 * n, *g2 = v + SV_S2 * n, *xb = v + SV_XB * n,
         *xz = v + SV_XZ * n, *rb = v + SV_RB * n, *rz = v + SV_RZ * n, *pb = v + SV_PB * n, *pz = v + SV_PZ * n,
         *qb = v + SV_QB * n, *qz = v + SV_QZ * n;

  // xi = A^T b_hat, lambda, the starting point beta = 0, z = |xi|_inf (1 if 0),
  // nu = lambda / 2 (reading "barrier strategy")
  at_apply<RMAX>(sig, obs, xi, d, T, w0, w1);
  double xinf = 0.0;
  for (long long f = threadIdx.x; f < n; f += kSmallThreads) xinf = fmax(xinf, fabs(xi[f]));
  xinf = block_reduce(xinf, 1, red);
  const double lam = lambdas ? lambdas[p] : lambda_frac * xinf;
  const double z0 = xinf > 0.0 ? xinf : 1.0;
  for (long long f = threadIdx.x; f < n; f += kSmallThreads) {
    be[f] = 0.0;
    zv[f] = z0;
    nu1[f] = 0.5 * lam;
    nu2[f] = 0.5 * lam;
  }
  __syncthreads();

  int it = 0, cg_total = 0, status = 1;   // 1: not converged (iteration limit)
  double rel = INFINITY, mu = 0.0;
  for (;; ++it) {
    // residual of the iterate (equation "kkt") and its relative size
    h_apply<RMAX>(be, hb, obs, d, T, w0, w1);
    double fb = 0.0, fz = 0.0, cmax = 0.0, csum = 0.0;
    bool bad = false;
    for (long long f = threadIdx.x; f < n; f += kSmallThreads) {
      const double s1 = zv[f] + be[f], s2 = zv[f] - be[f];
      const double a = hb[f] - xi[f] - nu1[f] + nu2[f];
      const double b = lam - nu1[f] - nu2[f];
      const double c1 = s1 * nu1[f], c2 = s2 * nu2[f];
      fb = fmax(fb, fabs(a));
      fz = fmax(fz, fabs(b));
      cmax = fmax(cmax, fmax(c1, c2));
      csum += c1 + c2;
      bad = bad || !isfinite(a) || !isfinite(c1) || !isfinite(c2);
    }
    fb = block_reduce(fb, 1, red);
    fz = block_reduce(fz, 1, red);
    cmax = block_reduce(cmax, 1, red);
    csum = block_reduce(csum, 0, red);
    const double nbad = block_reduce(bad ? 1.0 : 0.0, 0, red);
    mu = csum / (2.0 * (double)n);
    rel = fmax(fmax(fb, fz), cmax) / (1.0 + xinf);
    if (nbad > 0.0) {
      status = -2;   // non-finite iterate
      break;
    }
    if (rel <= o.tol) {
      status = 0;
      break;
    }
    if (it >= o.max_iter) break;

    // Newton system (equation "condensedkkt"): Sigma_j = nu_j / s_j and the
    // right-hand side from equation "kktmu" (reading "Newton RHS"), in r;
    // PCG from x = 0 on K with the paper's P
    const double smu = o.sigma * mu;
    const double eta = fmin(o.cg_rtol, 0.1 * rel);
    double rho = 0.0;
    for (long long f = threadIdx.x; f < n; f += kSmallThreads) {
      const double s1 = zv[f] + be[f], s2 = zv[f] - be[f];
      const double i1 = 1.0 / s1, i2 = 1.0 / s2;
      const double a1 = nu1[f] * i1, a2 = nu2[f] * i2;
      g1[f] = a1;
      g2[f] = a2;
      const double r1 = -(hb[f] - xi[f]) + smu * (i1 - i2);
      const double r2 = -lam + smu * (i1 + i2);
      rb[f] = r1;
      rz[f] = r2;
      xb[f] = 0.0;
      xz[f] = 0.0;
      double w1v, w2v;
      pinv1(r1, r2, a1, a2, w1v, w2v);
      pb[f] = w1v;
      pz[f] = w2v;
      rho += r1 * w1v + r2 * w2v;
    }
    rho = block_reduce(rho, 0, red);
    const double tol = fmax(o.cg_atol, eta * sqrt(fmax(rho, 0.0)));
    int cg = 0;
    while (sqrt(fmax(rho, 0.0)) > tol && cg < o.cg_max) {
      // q = K p (H p_beta plus the Sigma terms)
      h_apply<RMAX>(pb, qb, obs, d, T, w0, w1);
      double pq = 0.0;
      for (long long f = threadIdx.x; f < n; f += kSmallThreads) {
        const double L1 = g1[f] + g2[f], L2 = g1[f] - g2[f];
        const double a = qb[f] + L1 * pb[f] + L2 * pz[f];
        const double b = L2 * pb[f] + L1 * pz[f];
        qb[f] = a;
        qz[f] = b;
        pq += pb[f] * a + pz[f] * b;
      }
      pq = block_reduce(pq, 0, red);
      const double alpha = rho / pq;
      double rn = 0.0;
      for (long long f = threadIdx.x; f < n; f += kSmallThreads) {
        xb[f] += alpha * pb[f];
        xz[f] += alpha * pz[f];
        const double r1 = rb[f] - alpha * qb[f], r2 = rz[f] - alpha * qz[f];
        rb[f] = r1;
        rz[f] = r2;
        double w1v, w2v;
        pinv1(r1, r2, g1[f], g2[f], w1v, w2v);
        qb[f] = w1v;   // z = P^{-1} r, kept in q until the direction update
        qz[f] = w2v;
        rn += r1 * w1v + r2 * w2v;
      }
      rn = block_reduce(rn, 0, red);
      const double bt = rn / rho;
      rho = rn;
      for (long long f = threadIdx.x; f < n; f += kSmallThreads) {
        pb[f] = qb[f] + bt * pb[f];
        pz[f] = qz[f] + bt * pz[f];
      }
      __syncthreads();
      ++cg;
    }
    cg_total += cg;

    // multiplier direction, step to the boundary and update
    double amax = INFINITY;
    for (long long f = threadIdx.x; f < n; f += kSmallThreads) {
      const double s1 = zv[f] + be[f], s2 = zv[f] - be[f];
      const double ds1 = xb[f] + xz[f], ds2 = xz[f] - xb[f];
      const double dn1 = smu / s1 - nu1[f] - g1[f] * ds1;
      const double dn2 = smu / s2 - nu2[f] - g2[f] * ds2;
      rb[f] = dn1;
      rz[f] = dn2;
      amax = fmin(amax, fmin(fmin(ratio(s1, ds1), ratio(s2, ds2)), fmin(ratio(nu1[f], dn1), ratio(nu2[f], dn2))));
    }
    amax = block_reduce(amax, 2, red);
    const double step = fmin(1.0, o.tau * amax);
    for (long long f = threadIdx.x; f < n; f += kSmallThreads) {
      be[f] += step * xb[f];
      zv[f] += step * xz[f];
      nu1[f] += step * rb[f];
      nu2[f] += step * rz[f];
    }
    __syncthreads();
  }
  for (long long f = threadIdx.x; f < n; f += kSmallThreads) beta_out[(long long)p * n + f] = be[f];
  if (threadIdx.x == 0) {
    double* out = info + (long long)p * CSIPM_SMALL_INFO;
    out[0] = (double)status;
    out[1] = (double)it;
    out[2] = (double)cg_total;
    out[3] = rel;
    out[4] = mu;
    out[5] = lam;
  }
}

}  // namespace

bool small_supported(int n1, int n2, int n3) {
  return n1 >= 1 && n2 >= 1 && n3 >= 1 && n1 <= kSmallMaxExtent && n2 <= kSmallMaxExtent &&
         n3 <= kSmallMaxExtent;
}

namespace {
// complex buffers of the transforms: the spectrum, and a scratch copy when
// an extent has no register pass
int spectrum_buffers(int n1, int n2, int n3) {
  const auto reg = [](int L) { return L == 1 || reg_length(L); };
  return reg(n1) && reg(n2) && reg(n3) ? 1 : 2;
}
bool spectrum_in_lds(int n1, int n2, int n3) {
  const long long n = (long long)n1 * n2 * n3;
  return (long long)spectrum_buffers(n1, n2, n3) * n * (long long)sizeof(cx<double>) <= kSmallLdsBytes;
}
}  // namespace

size_t small_problem_bytes(int n1, int n2, int n3) {
  const long long n = (long long)n1 * n2 * n3;
  const bool lds = spectrum_in_lds(n1, n2, n3);
  // SV_COUNT real arrays, and the spectrum buffers when they do not sit in LDS
  size_t b = sizeof(double) * (size_t)n * (size_t)SV_COUNT +
             (lds ? 0 : (size_t)spectrum_buffers(n1, n2, n3) * sizeof(cx<double>) * (size_t)n);
  return (b + 255) & ~(size_t)255;
}

hipError_t small_launch(int n1, int n2, int n3, int count, const double* signals, const uint8_t* observed,
                        const double* lambdas, double lambda_frac, double* beta_out, double* info, char* ws,
                        const cx<double>* tw, const SmallOpts& o, hipStream_t s) {
  const long long n = (long long)n1 * n2 * n3;
  const bool lds = spectrum_in_lds(n1, n2, n3);
  const size_t shm = lds ? (size_t)spectrum_buffers(n1, n2, n3) * sizeof(cx<double>) * (size_t)n : 0;
  const bool has32 = n1 == 32 || n2 == 32 || n3 == 32;
  const void* kern = has32 ? (const void*)k_small_solve<32> : (const void*)k_small_solve<16>;
  if (shm > 65536) {
    const hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  const long long stride = (long long)small_problem_bytes(n1, n2, n3);
  if (has32)
    hipLaunchKernelGGL(k_small_solve<32>, dim3(count), dim3(kSmallThreads), shm, s, n1, n2, n3, signals, observed,
                       lambdas, lambda_frac, beta_out, info, ws, stride, tw, o, lds ? 1 : 0);
  else
    hipLaunchKernelGGL(k_small_solve<16>, dim3(count), dim3(kSmallThreads), shm, s, n1, n2, n3, signals, observed,
                       lambdas, lambda_frac, beta_out, info, ws, stride, tw, o, lds ? 1 : 0);
  return hipGetLastError();
}

}  // namespace csipm

using csipm::cx;

extern "C" size_t csipm_small_workspace_bytes(int n1, int n2, int n3, int count) {
  if (!csipm::small_supported(n1, n2, n3) || count < 1) return 0;
  const size_t tw = (sizeof(cx<double>) * (size_t)(n1 + n2 + n3) + 255) & ~(size_t)255;
  return tw + (size_t)count * csipm::small_problem_bytes(n1, n2, n3);
}

extern "C" csipm_status csipm_solve_small_batch(int n1, int n2, int n3, int count, const double* d_signals,
                                                const uint8_t* d_observed, const double* d_lambdas,
                                                double lambda_frac, const csipm_options* opts, double* d_beta_out,
                                                double* d_info, void* d_workspace, size_t workspace_bytes,
                                                void* hip_stream) {
  if (count < 1 || !d_signals || !d_observed || !opts || !d_beta_out || !d_info || !d_workspace ||
      (!d_lambdas && !(lambda_frac > 0.0 && std::isfinite(lambda_frac)))) {
    csipm::noctx_set_error("solve_small_batch: bad argument");
    return CSIPM_EINVAL;
  }
  if ((reinterpret_cast<uintptr_t>(d_workspace) & 255) != 0) {
    csipm::noctx_set_error("solve_small_batch: workspace not 256-byte aligned");
    return CSIPM_EINVAL;
  }
  if (!csipm::small_supported(n1, n2, n3)) {
    csipm::noctx_set_error("solve_small_batch: extents must lie in [1, 64]");
    return CSIPM_EUNSUPPORTED;
  }
  if (!(opts->tol > 0.0) || opts->max_iter < 0 || opts->cg_max < 0 || !(opts->tau > 0.0 && opts->tau < 1.0) ||
      !(opts->sigma > 0.0 && opts->sigma <= 1.0) || !(opts->cg_rtol >= 0.0) || !(opts->cg_atol >= 0.0)) {
    csipm::noctx_set_error("solve_small_batch: options out of range");
    return CSIPM_EINVAL;
  }
  const size_t need = csipm_small_workspace_bytes(n1, n2, n3, count);
  if (workspace_bytes < need) {
    csipm::noctx_set_error("solve_small_batch: workspace smaller than csipm_small_workspace_bytes");
    return CSIPM_ENOMEM;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  // twiddle tables exp(-2 pi i q / L) for L = n1, n2, n3, from long double
  // rounded once, at the front of the workspace
  std::vector<cx<double>> h;
  for (int L : {n1, n2, n3})
    for (int q = 0; q < L; ++q) {
      const long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)q / (long double)L;
      h.push_back({(double)cosl(a), (double)sinl(a)});
    }
  char* ws = reinterpret_cast<char*>(d_workspace);
  hipError_t e = hipMemcpyAsync(ws, h.data(), h.size() * sizeof(cx<double>), hipMemcpyHostToDevice, s);
  // (the host vector must outlive the copy)
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const size_t tw = (sizeof(cx<double>) * h.size() + 255) & ~(size_t)255;
  const csipm::SmallOpts o{opts->tol, opts->max_iter, opts->cg_max, opts->cg_rtol, opts->cg_atol, opts->sigma,
                           opts->tau};
  if (e == hipSuccess)
    e = csipm::small_launch(n1, n2, n3, count, d_signals, d_observed, d_lambdas, lambda_frac, d_beta_out, d_info,
                            ws + tw, reinterpret_cast<const cx<double>*>(ws), o, s);
  if (e != hipSuccess) {
    csipm::noctx_set_error(std::string("solve_small_batch: ") + hipGetErrorString(e));
    return CSIPM_EHIP;
  }
  return CSIPM_OK;
}
