// Elementwise kernels of the Krylov solver and the interior-point method,
// each fused with the reductions it needs (paper: sections "Primal-dual
// interior-point method", "Condensed KKT system", "Krylov methods and
// preconditioners").  Every reduction is two-stage and deterministic: a fixed
// grid writes one partial per workgroup, then a single-workgroup finalize
// kernel combines the partials in a fixed order and applies the scalar logic
// (alpha, beta, stopping test) on the device.
#include "vec.h"

#include <cmath>
#include <type_traits>

namespace csipm {

namespace {


// Block (256 threads) reduction of NQ values with per-value op; thread 0
// writes out[q * stride + blockIdx.x].
template <int NQ>
__device__ __forceinline__ void block_reduce_store(double* v, const int* ops, double* out, int stride) {
  __shared__ double red[NQ][4];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double x = v[q];
    x = ops[q] == RED_SUM ? wave_sum(x) : ops[q] == RED_MAX ? wave_max(x) : wave_min(x);
    if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double x = red[q][0];
      for (int w = 1; w < 4; ++w)
        x = ops[q] == RED_SUM ? x + red[q][w] : ops[q] == RED_MAX ? fmax(x, red[q][w]) : fmin(x, red[q][w]);
      out[q * stride + blockIdx.x] = x;
    }
  }
}

__device__ __forceinline__ double block_sum_256(double v) {
  __shared__ double red[4];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return s;
}

template <typename T>
__device__ __forceinline__ void pinv1(T rb, T rz, T s1, T s2, double c, T& zb, T& zz) {
  pinv_block<T>(rb, rz, s1, s2, c, zb, zz);
}

__device__ __forceinline__ long long gtid() { return blockIdx.x * (long long)blockDim.x + threadIdx.x; }
__device__ __forceinline__ long long gstride() { return (long long)gridDim.x * blockDim.x; }

// Elementwise loops visit pairs of neighbouring elements (n is even) from
// pointers known to be 2-element aligned, so each lane moves 16 bytes per
// FP64 array per access.
#define CSIPM_PAIRS(n)                                                      \
  for (long long j_ = gtid(); j_ < (n) / 2; j_ += gstride())                \
    _Pragma("unroll") for (long long i = 2 * j_; i < 2 * j_ + 2; ++i)
#define CSIPM_ALIGN(p) p = (decltype(p))__builtin_assume_aligned(p, 2 * sizeof(*(p)))

// ------------------------------------------------------------------- PCG --
// x += alpha p (x = alpha p on the first iteration: x0 = 0 is never stored),
// r -= alpha q, z = P_c^{-1} r, partial r.z.  A first iteration of a solve
// that finished at initialisation writes x = 0 and nothing else.
template <typename T>
__global__ void __launch_bounds__(256)
k_cg_update(T* __restrict__ xb, T* __restrict__ xz, const T* __restrict__ pb, const T* __restrict__ pz,
            const T* __restrict__ qb, const T* __restrict__ qz, T* __restrict__ rb, T* __restrict__ rz,
            T* __restrict__ zb, T* __restrict__ zz, const T* __restrict__ s1, const T* __restrict__ s2,
            const float* __restrict__ c, const double* __restrict__ scal, const int* __restrict__ flags,
            long long n, double* partial, int first) {
  CSIPM_ALIGN(xb);
  CSIPM_ALIGN(xz);
  CSIPM_ALIGN(pb);
  CSIPM_ALIGN(pz);
  CSIPM_ALIGN(qb);
  CSIPM_ALIGN(qz);
  CSIPM_ALIGN(rb);
  CSIPM_ALIGN(rz);
  CSIPM_ALIGN(zb);
  CSIPM_ALIGN(zz);
  CSIPM_ALIGN(s1);
  CSIPM_ALIGN(s2);

  if (flags[F_DONE]) {
    if (first)
      CSIPM_PAIRS(n) {
        xb[i] = T(0);
        xz[i] = T(0);
      }
    return;
  }
  const T a = (T)scal[S_ALPHA];
  double acc = 0.0;
  using V = cx<T>;
  const V *PB = (const V*)pb, *PZ = (const V*)pz, *QB = (const V*)qb, *QZ = (const V*)qz, *S1 = (const V*)s1,
          *S2 = (const V*)s2;
  V *XB = (V*)xb, *XZ = (V*)xz, *RB = (V*)rb, *RZ = (V*)rz, *ZB = (V*)zb, *ZZ = (V*)zz;
  const float2* C2 = (const float2*)c;
  for (long long j = gtid(); j < n / 2; j += gstride()) {
    const V p1 = PB[j], p2 = PZ[j];
    V x1, x2;
    if (first) {
      x1 = {a * p1.re, a * p1.im};
      x2 = {a * p2.re, a * p2.im};
    } else {
      x1 = XB[j];
      x2 = XZ[j];
      x1 = {x1.re + a * p1.re, x1.im + a * p1.im};
      x2 = {x2.re + a * p2.re, x2.im + a * p2.im};
    }
    XB[j] = x1;
    XZ[j] = x2;
    const V q1 = QB[j], q2 = QZ[j], r1 = RB[j], r2 = RZ[j];
    const V b = {r1.re - a * q1.re, r1.im - a * q1.im};
    const V z = {r2.re - a * q2.re, r2.im - a * q2.im};
    RB[j] = b;
    RZ[j] = z;
    const V g1 = S1[j], g2 = S2[j];
    const float2 cc = C2 ? C2[j] : make_float2(1.0f, 1.0f);
    V ub, uz;
    pinv1<T>(b.re, z.re, g1.re, g2.re, (double)cc.x, ub.re, uz.re);
    pinv1<T>(b.im, z.im, g1.im, g2.im, (double)cc.y, ub.im, uz.im);
    ZB[j] = ub;
    ZZ[j] = uz;
    acc += (double)b.re * (double)ub.re + (double)z.re * (double)uz.re + (double)b.im * (double)ub.im +
           (double)z.im * (double)uz.im;
  }
  const int op = RED_SUM;
  block_reduce_store<1>(&acc, &op, partial, 0);
}

// Conjugate residuals, direction step: p = z + beta p and q = w + beta q
// (p = z, q = w on the first iteration), where w = K z came from the
// K-apply; partial sums of q.P_c^{-1}q, the denominator of alpha.
template <typename T>
__global__ void __launch_bounds__(256)
k_cr_dir(T* __restrict__ pb, T* __restrict__ pz, T* __restrict__ qb, T* __restrict__ qz,
         const T* __restrict__ zb, const T* __restrict__ zz, const T* __restrict__ wb, const T* __restrict__ wz,
         const T* __restrict__ s1, const T* __restrict__ s2, const float* __restrict__ c,
         const double* __restrict__ scal, const int* __restrict__ flags, long long n, double* partial, int first) {
  CSIPM_ALIGN(pb);
  CSIPM_ALIGN(pz);
  CSIPM_ALIGN(qb);
  CSIPM_ALIGN(qz);
  CSIPM_ALIGN(zb);
  CSIPM_ALIGN(zz);
  CSIPM_ALIGN(wb);
  CSIPM_ALIGN(wz);
  CSIPM_ALIGN(s1);
  CSIPM_ALIGN(s2);

  if (flags[F_DONE]) return;
  const T be = first ? T(0) : (T)scal[S_BETA];
  double acc = 0.0;
  CSIPM_PAIRS(n) {
    const T p1 = first ? zb[i] : zb[i] + be * pb[i];
    const T p2 = first ? zz[i] : zz[i] + be * pz[i];
    const T q1 = first ? wb[i] : wb[i] + be * qb[i];
    const T q2 = first ? wz[i] : wz[i] + be * qz[i];
    pb[i] = p1;
    pz[i] = p2;
    qb[i] = q1;
    qz[i] = q2;
    T u1, u2;
    pinv1<T>(q1, q2, s1[i], s2[i], c ? (double)c[i] : 1.0, u1, u2);
    acc += (double)q1 * (double)u1 + (double)q2 * (double)u2;
  }
  const int op = RED_SUM;
  block_reduce_store<1>(&acc, &op, partial, 0);
}

// Conjugate A-residuals (CAr), in the P_c^{-1} space: z = P^{-1} r,
// u = P^{-1} K z, v = P^{-1} K p and y = P^{-1} K v are kept, r = P z and
// the other K images are implied.  Direction step after s = K u:
// p = z + beta p, v = u + beta v, y = P^{-1}s + beta y (p = z, v = u,
// y = P^{-1}s first); partial sums of y.(P y), the denominator of alpha.
template <typename T>
__global__ void __launch_bounds__(256)
k_car_dir(T* __restrict__ pb, T* __restrict__ pz, T* __restrict__ vb, T* __restrict__ vz, T* __restrict__ yb,
          T* __restrict__ yz, const T* __restrict__ zb, const T* __restrict__ zz, const T* __restrict__ ub,
          const T* __restrict__ uz, const T* __restrict__ sb, const T* __restrict__ sz, const T* __restrict__ s1,
          const T* __restrict__ s2, const float* __restrict__ c, const double* __restrict__ scal,
          const int* __restrict__ flags, long long n, double* partial, int first) {
  CSIPM_ALIGN(pb);
  CSIPM_ALIGN(pz);
  CSIPM_ALIGN(vb);
  CSIPM_ALIGN(vz);
  CSIPM_ALIGN(yb);
  CSIPM_ALIGN(yz);
  CSIPM_ALIGN(zb);
  CSIPM_ALIGN(zz);
  CSIPM_ALIGN(ub);
  CSIPM_ALIGN(uz);
  CSIPM_ALIGN(sb);
  CSIPM_ALIGN(sz);
  CSIPM_ALIGN(s1);
  CSIPM_ALIGN(s2);

  if (flags[F_DONE]) return;
  const T be = first ? T(0) : (T)scal[S_BETA];
  double acc = 0.0;
  CSIPM_PAIRS(n) {
    const double cc = c ? (double)c[i] : 1.0;
    T h1, h2;
    pinv1<T>(sb[i], sz[i], s1[i], s2[i], cc, h1, h2);
    const T p1 = first ? zb[i] : zb[i] + be * pb[i];
    const T p2 = first ? zz[i] : zz[i] + be * pz[i];
    const T v1 = first ? ub[i] : ub[i] + be * vb[i];
    const T v2 = first ? uz[i] : uz[i] + be * vz[i];
    const T y1 = first ? h1 : h1 + be * yb[i];
    const T y2 = first ? h2 : h2 + be * yz[i];
    pb[i] = p1;
    pz[i] = p2;
    vb[i] = v1;
    vz[i] = v2;
    yb[i] = y1;
    yz[i] = y2;
    double t1, t2;
    p_block<T>(y1, y2, s1[i], s2[i], cc, t1, t2);
    acc += (double)y1 * t1 + (double)y2 * t2;
  }
  const int op = RED_SUM;
  block_reduce_store<1>(&acc, &op, partial, 0);
}

// CAr update: x += alpha p (x = alpha p first), z -= alpha v, u -= alpha y;
// partial sums of z.(P z) = r.P^{-1}r, the stopping norm.  A first
// iteration of a solve that finished at initialisation writes x = 0.
template <typename T>
__global__ void __launch_bounds__(256)
k_car_update(T* __restrict__ xb, T* __restrict__ xz, const T* __restrict__ pb, const T* __restrict__ pz,
             T* __restrict__ zb, T* __restrict__ zz, const T* __restrict__ vb, const T* __restrict__ vz,
             T* __restrict__ ub, T* __restrict__ uz, const T* __restrict__ yb, const T* __restrict__ yz,
             const T* __restrict__ s1, const T* __restrict__ s2, const float* __restrict__ c,
             const double* __restrict__ scal, const int* __restrict__ flags, long long n, double* partial,
             int first) {
  CSIPM_ALIGN(xb);
  CSIPM_ALIGN(xz);
  CSIPM_ALIGN(pb);
  CSIPM_ALIGN(pz);
  CSIPM_ALIGN(zb);
  CSIPM_ALIGN(zz);
  CSIPM_ALIGN(vb);
  CSIPM_ALIGN(vz);
  CSIPM_ALIGN(ub);
  CSIPM_ALIGN(uz);
  CSIPM_ALIGN(yb);
  CSIPM_ALIGN(yz);
  CSIPM_ALIGN(s1);
  CSIPM_ALIGN(s2);

  if (flags[F_DONE]) {
    if (first)
      CSIPM_PAIRS(n) {
        xb[i] = T(0);
        xz[i] = T(0);
      }
    return;
  }
  const T a = (T)scal[S_ALPHA];
  double acc = 0.0;
  CSIPM_PAIRS(n) {
    xb[i] = first ? a * pb[i] : xb[i] + a * pb[i];
    xz[i] = first ? a * pz[i] : xz[i] + a * pz[i];
    const T z1 = zb[i] - a * vb[i], z2 = zz[i] - a * vz[i];
    zb[i] = z1;
    zz[i] = z2;
    ub[i] = ub[i] - a * yb[i];
    uz[i] = uz[i] - a * yz[i];
    double r1, r2;
    p_block<T>(z1, z2, s1[i], s2[i], c ? (double)c[i] : 1.0, r1, r2);
    acc += (double)z1 * r1 + (double)z2 * r2;
  }
  const int op = RED_SUM;
  block_reduce_store<1>(&acc, &op, partial, 0);
}

// r = P_c z: the residual of a CAr solve, which keeps only z = P^{-1} r,
// for the interior-point update that recovers H d_beta from it.
template <typename T>
__global__ void __launch_bounds__(256)
k_p_apply(const T* __restrict__ zb, const T* __restrict__ zz, const T* __restrict__ s1, const T* __restrict__ s2,
          const float* __restrict__ c, T* __restrict__ rb, T* __restrict__ rz, long long n) {
  CSIPM_ALIGN(zb);
  CSIPM_ALIGN(zz);
  CSIPM_ALIGN(s1);
  CSIPM_ALIGN(s2);
  CSIPM_ALIGN(rb);
  CSIPM_ALIGN(rz);
  CSIPM_PAIRS(n) {
    double r1, r2;
    p_block<T>(zb[i], zz[i], s1[i], s2[i], c ? (double)c[i] : 1.0, r1, r2);
    rb[i] = (T)r1;
    rz[i] = (T)r2;
  }
}

__device__ __forceinline__ double fin_sum(const double* partial, int nb) {
  double a = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) a += partial[i];
  return block_sum_256(a);
}

// Starts a PCG solve: rz0 from the partials (quantity 0) or, when
// from_slot >= 0, from scal[from_slot]; with ref_slot >= 0 the second
// quantity of the partials is summed into scal[ref_slot].
__global__ void __launch_bounds__(256)
k_fin_cg_init(const double* partial, int nb, int stride, double* scal, int* flags, double eta, double atol,
              int maxit, int ref_slot, int from_slot) {
  const double rzp = from_slot >= 0 ? 0.0 : fin_sum(partial, nb);
  const double ref = ref_slot >= 0 ? fin_sum(partial + stride, nb) : 0.0;
  if (threadIdx.x == 0) {
    const double rz0 = from_slot >= 0 ? scal[from_slot] : rzp;
    if (ref_slot >= 0) scal[ref_slot] = ref;
    scal[S_RZ] = rz0;
    scal[S_RZ0] = rz0;
    const double r0 = sqrt(fmax(rz0, 0.0));
    const double tol = fmax(atol, eta * r0);
    scal[S_TOL] = tol;
    scal[S_RES] = r0;
    flags[F_IT] = 0;
    flags[F_BREAK] = 0;
    flags[F_DONE] = (r0 <= tol || maxit <= 0 || !(rz0 == rz0)) ? 1 : 0;
    flags[F_MAXIT] = maxit;
  }
}

__global__ void __launch_bounds__(256)
k_fin_alpha(const double* partial, int nb, double* scal, int* flags) {
  if (flags[F_DONE]) return;
  const double pq = fin_sum(partial, nb);
  if (threadIdx.x == 0) {
    scal[S_PQ] = pq;
    if (!(pq > 0.0) || !isfinite(pq)) {
      // loss of positive definiteness in floating point: stop the solve
      scal[S_ALPHA] = 0.0;
      flags[F_BREAK] = 1;
      flags[F_DONE] = 1;
    } else {
      scal[S_ALPHA] = scal[S_RZ] / pq;
    }
  }
}

__global__ void __launch_bounds__(256)
k_fin_rz(const double* partial, int nb, double* scal, int* flags) {
  if (flags[F_DONE]) return;
  const double rz = fin_sum(partial, nb);
  if (threadIdx.x == 0) {
    scal[S_BETA] = rz / scal[S_RZ];
    scal[S_RZ] = rz;
    const double r = sqrt(fmax(rz, 0.0));
    scal[S_RES] = r;
    const int it = flags[F_IT] + 1;
    flags[F_IT] = it;
    flags[F_DONE] = (r <= scal[S_TOL] || it >= flags[F_MAXIT] || !isfinite(rz)) ? 1 : 0;
  }
}

// Conjugate residuals, after w = K z: beta = (z.w) / (z.w)_previous (not on
// the first iteration), and S_RZ = z.w, the numerator of alpha.  A
// non-positive or non-finite z.w ends the solve.
__global__ void __launch_bounds__(256)
k_fin_cr_zw(const double* partial, int nb, double* scal, int* flags, int first) {
  if (flags[F_DONE]) return;
  const double zw = fin_sum(partial, nb);
  if (threadIdx.x == 0) {
    if (!(zw > 0.0) || !isfinite(zw)) {
      flags[F_BREAK] = 1;
      flags[F_DONE] = 1;
      return;
    }
    if (!first) scal[S_BETA] = zw / scal[S_ZW];
    scal[S_ZW] = zw;
    scal[S_RZ] = zw;
  }
}

// ------------------------------------------------------------------- IPM --
__global__ void __launch_bounds__(256)
k_ipm_init(double* __restrict__ beta, double* __restrict__ z, double* __restrict__ nu1, double* __restrict__ nu2,
           double* __restrict__ g, const double* __restrict__ xi, long long n, double z0, double lam) {
  for (long long i = gtid(); i < n; i += gstride()) {
    beta[i] = 0.0;
    g[i] = -xi[i];
    z[i] = z0;
    nu1[i] = 0.5 * lam;
    nu2[i] = 0.5 * lam;
  }
}

// Residual parts of the KKT system (equation "kkt", first two rows) and
// complementarity: [max|F_b|, max|F_z|, max s.nu, sum s.nu, max|beta|,
// min(s, nu), count of non-finite values, sum log(S1 + S2) (when logsum is
// set: the centring of the learned correction's first feature)].
constexpr int NRESID = NRESID_Q;
#define CSIPM_RESID_OPS \
  {RED_MAX, RED_MAX, RED_MAX, RED_SUM, RED_MAX, RED_MIN, RED_SUM, RED_SUM, RED_SUM, RED_MAX}
#define CSIPM_RESID_OPS_NI \
  {RED_MAX, RED_MAX, RED_MAX, RED_SUM, RED_MAX, RED_MIN, RED_SUM, RED_SUM, RED_SUM, RED_MAX, RED_SUM, RED_SUM}

__device__ __forceinline__ void resid_accumulate(double* v, double b, double s1, double s2, double a1, double a2,
                                                 double fb, double fz, int logsum) {
  const double c1 = s1 * a1, c2 = s2 * a2;
  v[0] = fmax(v[0], fabs(fb));
  v[1] = fmax(v[1], fabs(fz));
  v[2] = fmax(v[2], fmax(c1, c2));
  v[3] += c1 + c2;
  v[4] = fmax(v[4], fabs(b));
  v[5] = fmin(v[5], fmin(fmin(s1, s2), fmin(a1, a2)));
  if (!isfinite(fb) || !isfinite(c1) || !isfinite(c2)) v[6] += 1.0;
  if (logsum) {
    v[7] += log(a1 / s1 + a2 / s2);
    // coefficients where the learned correction can matter
    v[8] += pc_gate(a1, a2, s1, s2) ? 1.0 : 0.0;
  }
}
__global__ void __launch_bounds__(256)
k_ipm_resid(const double* __restrict__ beta, const double* __restrict__ z, const double* __restrict__ nu1,
            const double* __restrict__ nu2, double* __restrict__ hb, const double* __restrict__ xi,
            double lam, long long n, double* partial, int stride, int logsum) {
  CSIPM_ALIGN(beta);
  CSIPM_ALIGN(z);
  CSIPM_ALIGN(nu1);
  CSIPM_ALIGN(nu2);
  CSIPM_ALIGN(hb);
  CSIPM_ALIGN(xi);

  double v[NRESID] = {0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, 0.0, 0.0, 0.0, 0.0};
  CSIPM_PAIRS(n) {
    const double b = beta[i], zz = z[i], a1 = nu1[i], a2 = nu2[i];
    const double s1 = zz + b, s2 = zz - b;
    double g = hb[i];
    if (xi) {   // hb holds H beta: keep G = H beta - xi from here on
      g -= xi[i];
      hb[i] = g;
    }
    const double fb = g - a1 + a2;
    const double fz = lam - a1 - a2;
    resid_accumulate(v, b, s1, s2, a1, a2, fb, fz, logsum);
  }
  const int ops[NRESID] = CSIPM_RESID_OPS;
  block_reduce_store<NRESID>(v, ops, partial, stride);
}

// Search direction of the multipliers at one coefficient, with the barrier
// diagonals re-formed from the state exactly as the Newton build forms them:
//   s1 = z + beta, s2 = z - beta, Sigma_j = nu_j / s_j,
//   ds1 = db + dz, ds2 = dz - db, dnu_j = smu/s_j - nu_j - Sigma_j ds_j.
// With a predictor-corrector step the complementarity rows carry the
// second-order term c_j = ds_j dnu_j of the affine direction (ca = c1, c2),
// and smu / s_j becomes (smu - c_j) / s_j.
struct IpmDir {
  double s1, s2, i1, i2, g1, g2, ds1, ds2, dn1, dn2;
};
__device__ __forceinline__ IpmDir ipm_dir(double b, double zz, double a1, double a2, double d1, double d2,
                                          double smu, double c1 = 0.0, double c2 = 0.0, bool corr = false) {
  IpmDir o;
  o.s1 = zz + b;
  o.s2 = zz - b;
  o.i1 = 1.0 / o.s1;
  o.i2 = 1.0 / o.s2;
  o.g1 = a1 * o.i1;
  o.g2 = a2 * o.i2;
  o.ds1 = d1 + d2;
  o.ds2 = d2 - d1;
  if (corr) {
    o.dn1 = (smu - c1) * o.i1 - a1 - o.g1 * o.ds1;
    o.dn2 = (smu - c2) * o.i2 - a2 - o.g2 * o.ds2;
  } else {
    o.dn1 = smu * o.i1 - a1 - o.g1 * o.ds1;
    o.dn2 = smu * o.i2 - a2 - o.g2 * o.ds2;
  }
  return o;
}
// Second-order terms c_j = ds_j dnu_j of the affine direction (da1, da2) at
// one coefficient (dnu_j = -nu_j - Sigma_j ds_j: target 0).
__device__ __forceinline__ void corr_terms(double b, double zz, double a1, double a2, double da1, double da2,
                                           double& c1, double& c2) {
  const IpmDir d = ipm_dir(b, zz, a1, a2, da1, da2, 0.0);
  c1 = d.ds1 * d.dn1;
  c2 = d.ds2 * d.dn2;
}

// The Newton system at pair j from the state (b, z, nu1, nu2, G) of its two
// coefficients: Sigma_j = nu_j / s_j, h (with the corrector terms c1, c2
// when corr), r = h in TC, z = P_c^{-1} r in TC; adds r.z and h.P_c^{-1}h
// (FP64) to acc[0], acc[1].
template <typename TC>
__device__ __forceinline__ void newton_pair(const NewtonOut<TC>& o, long long j, const double* bb, const double* zz2,
                                            const double* n1, const double* n2, const double* hv, const double* cv,
                                            double lam, double smu, bool corr, const double* c1v, const double* c2v,
                                            double* acc) {
  using D2 = cx<double>;
  using V = cx<TC>;
  double g1o[2], g2o[2], h1o[2], h2o[2];
  TC r1o[2], r2o[2], w1o[2], w2o[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double s1 = zz2[k] + bb[k], s2 = zz2[k] - bb[k];
    const double i1 = 1.0 / s1, i2 = 1.0 / s2;
    const double g1 = n1[k] * i1, g2 = n2[k] * i2;
    double h1, h2;
    if (corr) {   // corrector of a predictor-corrector step
      const double u1 = (smu - c1v[k]) * i1, u2 = (smu - c2v[k]) * i2;
      h1 = -hv[k] + (u1 - u2);
      h2 = -lam + (u1 + u2);
    } else {
      h1 = -hv[k] + smu * (i1 - i2);
      h2 = -lam + smu * (i1 + i2);
    }
    double u1, u2;
    pinv_block<double>(h1, h2, g1, g2, cv[k], u1, u2);
    acc[1] += h1 * u1 + h2 * u2;
    const TC r1 = (TC)h1, r2 = (TC)h2;
    TC w1, w2;
    if constexpr (std::is_same<TC, double>::value) {
      w1 = u1;
      w2 = u2;
    } else {
      pinv_block<TC>(r1, r2, (TC)g1, (TC)g2, cv[k], w1, w2);
    }
    acc[0] += (double)r1 * (double)w1 + (double)r2 * (double)w2;
    g1o[k] = g1; g2o[k] = g2; h1o[k] = h1; h2o[k] = h2;
    r1o[k] = r1; r2o[k] = r2; w1o[k] = w1; w2o[k] = w2;
  }
  if (o.sig1) {
    ((D2*)o.sig1)[j] = {g1o[0], g1o[1]};
    ((D2*)o.sig2)[j] = {g2o[0], g2o[1]};
  }
  if (o.hb_out) {
    ((D2*)o.hb_out)[j] = {h1o[0], h1o[1]};
    ((D2*)o.hz_out)[j] = {h2o[0], h2o[1]};
  }
  if constexpr (!std::is_same<TC, double>::value) {
    ((V*)o.sig1c)[j] = {(TC)g1o[0], (TC)g1o[1]};
    ((V*)o.sig2c)[j] = {(TC)g2o[0], (TC)g2o[1]};
  }
  ((V*)o.rb)[j] = {r1o[0], r1o[1]};
  ((V*)o.rz)[j] = {r2o[0], r2o[1]};
  if (o.zb) {
    ((V*)o.zb)[j] = {w1o[0], w1o[1]};
    ((V*)o.zz)[j] = {w2o[0], w2o[1]};
  }
  ((V*)o.pb)[j] = {w1o[0], w1o[1]};
  ((V*)o.pz)[j] = {w2o[0], w2o[1]};
}

// Newton system and PCG start in one pass: Sigma_j = nu_j / s_j (FP64 when
// sig1 is set, and in TC when sig1c is set), the right-hand side h (written
// only when hb_out is set), r = h, z = P_c^{-1} r, p = z in the Krylov precision TC, and the
// partial sums r.z (in TC) and h.P_c^{-1}h (in FP64).  x0 = 0 is implicit.
template <typename TC, bool CORR>
__global__ void __launch_bounds__(256)
k_newton_init(const double* __restrict__ beta, const double* __restrict__ z, const double* __restrict__ nu1,
              const double* __restrict__ nu2, const double* __restrict__ hb, double lam, double smu,
              double* __restrict__ sig1, double* __restrict__ sig2, double* __restrict__ hb_out, double* __restrict__ hz_out, TC* __restrict__ sig1c,
              TC* __restrict__ sig2c, const float* __restrict__ c, TC* __restrict__ rb, TC* __restrict__ rz,
              TC* __restrict__ zb, TC* __restrict__ zz, TC* __restrict__ pb, TC* __restrict__ pz, long long n,
              double* partial, const double* __restrict__ dab, const double* __restrict__ daz) {
  CSIPM_ALIGN(beta);
  CSIPM_ALIGN(z);
  CSIPM_ALIGN(nu1);
  CSIPM_ALIGN(nu2);
  CSIPM_ALIGN(hb);
  CSIPM_ALIGN(sig1);
  CSIPM_ALIGN(sig2);
  CSIPM_ALIGN(rb);
  CSIPM_ALIGN(rz);
  CSIPM_ALIGN(zb);
  CSIPM_ALIGN(zz);
  CSIPM_ALIGN(pb);
  CSIPM_ALIGN(pz);

  double acc[2] = {0.0, 0.0};
  using D2 = cx<double>;
  const D2 *BE = (const D2*)beta, *ZV = (const D2*)z, *N1 = (const D2*)nu1, *N2 = (const D2*)nu2,
           *HB = (const D2*)hb;
  const float2* C2 = (const float2*)c;
  const NewtonOut<TC> o{sig1, sig2, hb_out, hz_out, sig1c, sig2c, rb, rz, zb, zz, pb, pz};
  for (long long j = gtid(); j < n / 2; j += gstride()) {
    const D2 b2 = BE[j], z2 = ZV[j], a1 = N1[j], a2 = N2[j], hh = HB[j];
    const float2 cc = C2 ? C2[j] : make_float2(1.0f, 1.0f);
    const double bb[2] = {b2.re, b2.im}, zz2[2] = {z2.re, z2.im}, n1[2] = {a1.re, a1.im},
                 n2[2] = {a2.re, a2.im}, hv[2] = {hh.re, hh.im}, cv[2] = {(double)cc.x, (double)cc.y};
    double c1v[2] = {0.0, 0.0}, c2v[2] = {0.0, 0.0};
    if constexpr (CORR) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
        corr_terms(bb[k], zz2[k], n1[k], n2[k], dab[2 * j + k], daz[2 * j + k], c1v[k], c2v[k]);
    }
    newton_pair<TC>(o, j, bb, zz2, n1, n2, hv, cv, lam, smu, CORR, c1v, c2v, acc);
  }
  const int ops[2] = {RED_SUM, RED_SUM};
  block_reduce_store<2>(acc, ops, partial, VEC_MAX_BLOCKS);
}

// Pair j of a Newton direction: from its FP32 copy when one is given (an
// FP32 solution taken without refinement), else from the FP64 array.
__device__ __forceinline__ cx<double> ld_dir(const cx<double>* d64, const float* d32, long long j) {
  if (d32) {
    const float2 f = reinterpret_cast<const float2*>(d32)[j];
    return {(double)f.x, (double)f.y};
  }
  return d64[j];
}

// Largest step keeping s and nu positive along (db, dz, dnu1, dnu2); with
// CORR (a corrector) dnu carries the affine direction's second-order terms;
// with DSDN also sum ds.dnu (quantity 1 of the partials: for the affine
// direction, mu at its step alpha is ((1 - alpha) s.nu + alpha^2 ds.dnu) /
// 2n); with MUSUM the sums s.dnu + nu.ds and ds.dnu (quantities 2 and 3)
// that give mu after the step.  (D32: the direction is read in FP32.)
template <bool D32, bool CORR, bool DSDN, bool MUSUM>
__global__ void __launch_bounds__(256)
k_ipm_ratio(const double* __restrict__ beta, const double* __restrict__ z, const double* __restrict__ nu1,
            const double* __restrict__ nu2, const double* __restrict__ db, const double* __restrict__ dz,
            const float* __restrict__ db32, const float* __restrict__ dz32, double smu, long long n,
            double* partial, const double* __restrict__ dab, const double* __restrict__ daz) {
  double v[4] = {INFINITY, 0.0, 0.0, 0.0};
  using D2 = cx<double>;
  for (long long j = gtid(); j < n / 2; j += gstride()) {
    const D2 b2 = ((const D2*)beta)[j], z2 = ((const D2*)z)[j], a1 = ((const D2*)nu1)[j], a2 = ((const D2*)nu2)[j],
             d1 = ld_dir((const D2*)db, D32 ? db32 : nullptr, j), d2 = ld_dir((const D2*)dz, D32 ? dz32 : nullptr, j);
    const double bb[2] = {b2.re, b2.im}, zv[2] = {z2.re, z2.im}, n1[2] = {a1.re, a1.im}, n2[2] = {a2.re, a2.im},
                 dbv[2] = {d1.re, d1.im}, dzv[2] = {d2.re, d2.im};
    double c1[2] = {0.0, 0.0}, c2[2] = {0.0, 0.0};
    if constexpr (CORR) {
      const D2 e1 = ((const D2*)dab)[j], e2 = ((const D2*)daz)[j];
      corr_terms(bb[0], zv[0], n1[0], n2[0], e1.re, e2.re, c1[0], c2[0]);
      corr_terms(bb[1], zv[1], n1[1], n2[1], e1.im, e2.im, c1[1], c2[1]);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const IpmDir d = ipm_dir(bb[k], zv[k], n1[k], n2[k], dbv[k], dzv[k], smu, c1[k], c2[k], CORR);
      if (d.ds1 < 0.0) v[0] = fmin(v[0], -d.s1 / d.ds1);
      if (d.ds2 < 0.0) v[0] = fmin(v[0], -d.s2 / d.ds2);
      if (d.dn1 < 0.0) v[0] = fmin(v[0], -n1[k] / d.dn1);
      if (d.dn2 < 0.0) v[0] = fmin(v[0], -n2[k] / d.dn2);
      if constexpr (DSDN) v[1] += d.ds1 * d.dn1 + d.ds2 * d.dn2;
      if constexpr (MUSUM) {   // s.nu after a step alpha: s.nu + alpha (s.dnu + nu.ds) + alpha^2 ds.dnu
        v[2] += d.s1 * d.dn1 + n1[k] * d.ds1 + d.s2 * d.dn2 + n2[k] * d.ds2;
        v[3] += d.ds1 * d.dn1 + d.ds2 * d.dn2;
      }
    }
  }
  if constexpr (MUSUM) {
    const int ops[4] = {RED_MIN, RED_SUM, RED_SUM, RED_SUM};
    block_reduce_store<4>(v, ops, partial, VEC_MAX_BLOCKS);
  } else if constexpr (DSDN) {
    const int ops[2] = {RED_MIN, RED_SUM};
    block_reduce_store<2>(v, ops, partial, VEC_MAX_BLOCKS);
  } else {
    const int op = RED_MIN;
    block_reduce_store<1>(v, &op, partial, 0);
  }
}

// Step length: scal[S_AMAX] and scal[S_ALPHA_IPM].  With musum (quantities 2
// and 3 of the ratio pass) also the next target scal[S_SMU] = sigma mu+ with
// mu+ = (s0 + alpha s1 + alpha^2 s2) / (2n) the duality measure after the step.
__global__ void __launch_bounds__(256)
k_fin_step(const double* partial, int nb, double tau, double* scal, int musum, double s0, double sigma,
           double inv2n) {
  double a = INFINITY, m1 = 0.0, m2 = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a = fmin(a, partial[i]);
    if (musum) {
      m1 += partial[2 * VEC_MAX_BLOCKS + i];
      m2 += partial[3 * VEC_MAX_BLOCKS + i];
    }
  }
  a = wave_min(a);
  m1 = wave_sum(m1);
  m2 = wave_sum(m2);
  __shared__ double red[3][4];
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = m1;
    red[2][threadIdx.x >> 6] = m2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double amax = fmin(fmin(red[0][0], red[0][1]), fmin(red[0][2], red[0][3]));
    const double alpha = fmin(1.0, tau * amax);
    scal[S_AMAX] = amax;
    scal[S_ALPHA_IPM] = alpha;
    if (musum) {
      const double s1 = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
      const double s2 = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
      scal[S_SMU] = sigma * fmax(0.0, s0 + alpha * s1 + alpha * alpha * s2) * inv2n;
    }
  }
}

// Step of the interior-point iterate by alpha = scal[S_ALPHA_IPM], with H beta
// carried along instead of recomputed: H beta += alpha H d_beta, where H d_beta
// is either given (hd, from the FP64 residual pass of the refinement) or
// recovered from the Krylov residual r = h - K d of the Newton system (rres in
// FP64, or rres32 from an FP32 solve taken without refinement),
//   H d_beta = h_beta - r_beta - Sigma_1 (d_beta + d_z) - Sigma_2 (d_beta - d_z)
// (the beta row of K in Sigma form).  The same pass reduces the residual parts
// of the new iterate in k_ipm_resid's order.  With NI it also builds the
// next Newton system from the new iterate (newton_pair, target scal[S_SMU],
// correction cn or none) and stores its r.z and h.P^{-1}h partials as
// quantities NRESID and NRESID + 1.  HDM selects the source of H d_beta:
// ADV_RRES64 (the FP64 Krylov residual), ADV_DIRECT (hd) or ADV_RRES32 (the
// FP32 residual, with the direction read in FP32); CORR adds the corrector
// terms of a predictor-corrector step.
enum { ADV_RRES64 = 0, ADV_DIRECT = 1, ADV_RRES32 = 2 };
template <typename TC, bool NI, int HDM, bool CORR>
__global__ void __launch_bounds__(256)
k_ipm_advance(double* __restrict__ beta, double* __restrict__ z, double* __restrict__ nu1, double* __restrict__ nu2,
              double* __restrict__ hbeta, const double* __restrict__ db,
              const double* __restrict__ dz, const double* __restrict__ hd, const double* rres,
              const float* rres32, const float* __restrict__ db32, const float* __restrict__ dz32,
              double lam, double smu, const double* __restrict__ scal, long long n, double* partial, int stride,
              int logsum, const double* __restrict__ dab, const double* __restrict__ daz, NewtonOut<TC> no,
              const float* __restrict__ cn, uint32_t* __restrict__ act) {
  const double a = scal[S_ALPHA_IPM];
  const double smu_next = NI ? scal[S_SMU] : 0.0;
  double v[NRESID + 2] = {0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  using D2 = cx<double>;
  D2 *BE = (D2*)beta, *ZV = (D2*)z, *N1 = (D2*)nu1, *N2 = (D2*)nu2, *HBV = (D2*)hbeta;
  const D2 *DB = (const D2*)db, *DZ = (const D2*)dz, *W = (const D2*)(HDM == ADV_DIRECT ? hd : rres);
  const float2* W32 = (const float2*)rres32;
  constexpr bool d32 = HDM == ADV_RRES32;
  for (long long j = gtid(); j < n / 2; j += gstride()) {
    const D2 b2 = BE[j], z2 = ZV[j], a1 = N1[j], a2 = N2[j], h2 = HBV[j];
    const D2 d1 = ld_dir(DB, d32 ? db32 : nullptr, j), d2 = ld_dir(DZ, d32 ? dz32 : nullptr, j);
    D2 w2;
    if constexpr (d32) {
      const float2 f = W32[j];
      w2 = {(double)f.x, (double)f.y};
    } else {
      w2 = W[j];
    }
    const double bb[2] = {b2.re, b2.im}, zv[2] = {z2.re, z2.im}, n1[2] = {a1.re, a1.im}, n2[2] = {a2.re, a2.im},
                 hv[2] = {h2.re, h2.im}, dbv[2] = {d1.re, d1.im},
                 dzv[2] = {d2.re, d2.im}, wv[2] = {w2.re, w2.im};
    double bo[2], zo[2], n1o[2], n2o[2], ho[2];
    double c1[2] = {0.0, 0.0}, c2[2] = {0.0, 0.0};
    if constexpr (CORR) {
      const D2 e1 = ((const D2*)dab)[j], e2 = ((const D2*)daz)[j];
      corr_terms(bb[0], zv[0], n1[0], n2[0], e1.re, e2.re, c1[0], c2[0]);
      corr_terms(bb[1], zv[1], n1[1], n2[1], e1.im, e2.im, c1[1], c2[1]);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const IpmDir d = ipm_dir(bb[k], zv[k], n1[k], n2[k], dbv[k], dzv[k], smu, c1[k], c2[k], CORR);
      double u;
      if constexpr (HDM == ADV_DIRECT) {
        u = wv[k];
      } else {
        const double hrhs = CORR ? -hv[k] + ((smu - c1[k]) * d.i1 - (smu - c2[k]) * d.i2) : -hv[k] + smu * (d.i1 - d.i2);
        u = (hrhs - wv[k]) - (d.g1 * (dbv[k] + dzv[k]) + d.g2 * (dbv[k] - dzv[k]));
        // rounding of the Sigma terms, here and in the Krylov recurrence
        // that produced r, scales like eps (S1 + S2)(|d_beta| + |d_z|)
        v[9] = fmax(v[9], (d.g1 + d.g2) * (fabs(dbv[k]) + fabs(dzv[k])));
      }
      const double b = bb[k] + a * dbv[k], zz = zv[k] + a * dzv[k];
      const double m1 = n1[k] + a * d.dn1, m2 = n2[k] + a * d.dn2;
      const double hb = hv[k] + a * u;
      bo[k] = b; zo[k] = zz; n1o[k] = m1; n2o[k] = m2; ho[k] = hb;
      resid_accumulate(v, b, zz + b, zz - b, m1, m2, hb - m1 + m2, lam - m1 - m2, logsum);
    }
    BE[j] = {bo[0], bo[1]};
    ZV[j] = {zo[0], zo[1]};
    N1[j] = {n1o[0], n1o[1]};
    N2[j] = {n2o[0], n2o[1]};
    HBV[j] = {ho[0], ho[1]};
    if (act) {
      // activity flags of the correction, one per 64 coefficients: the 64
      // lanes of a wave hold 64 consecutive pairs, i.e. two chunks
      const bool a = pc_gate(n1o[0], n2o[0], zo[0] + bo[0], zo[0] - bo[0]) ||
                     pc_gate(n1o[1], n2o[1], zo[1] + bo[1], zo[1] - bo[1]);
      const unsigned long long m = __ballot(a);
      const int lane = threadIdx.x & 63;
      if (lane == 0) act[j >> 5] = (m & 0xffffffffull) ? 1u : 0u;
      if (lane == 32) act[j >> 5] = (m >> 32) ? 1u : 0u;
    }
    if constexpr (NI) {
      const float2 cc = cn ? reinterpret_cast<const float2*>(cn)[j] : make_float2(1.0f, 1.0f);
      const double cv[2] = {(double)cc.x, (double)cc.y}, zero[2] = {0.0, 0.0};
      // (the r written here may be rres / rres32 itself: pair j was read above)
      newton_pair<TC>(no, j, bo, zo, n1o, n2o, ho, cv, lam, smu_next, false, zero, zero, v + NRESID);
    }
  }
  if constexpr (NI) {
    const int ops[NRESID + 2] = CSIPM_RESID_OPS_NI;
    block_reduce_store<NRESID + 2>(v, ops, partial, stride);
  } else {
    const int ops[NRESID] = CSIPM_RESID_OPS;
    block_reduce_store<NRESID>(v, ops, partial, stride);
  }
}

// Generic multi-value finalize: out[q] = op_q over partial[q*stride + 0..nb);
// all quantities are reduced in one sweep.
// one block of kFinThreads: at most two partials per thread and quantity for
// the VEC_MAX_BLOCKS partials of a vector pass, loaded before they are combined
constexpr int kFinThreads = 1024;
template <int NQ>
__global__ void __launch_bounds__(kFinThreads)
k_fin_reduce(const double* partial, int nb, int stride, double* out, RedOps<NQ> ops) {
  double a[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) a[q] = ops.op[q] == RED_SUM ? 0.0 : ops.op[q] == RED_MAX ? -INFINITY : INFINITY;
  for (int i = threadIdx.x; i < nb; i += kFinThreads) {
    double x[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) x[q] = partial[q * stride + i];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      a[q] = ops.op[q] == RED_SUM ? a[q] + x[q] : ops.op[q] == RED_MAX ? fmax(a[q], x[q]) : fmin(a[q], x[q]);
  }
  constexpr int W = kFinThreads / 64;
  __shared__ double red[NQ][W];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double x = ops.op[q] == RED_SUM ? wave_sum(a[q]) : ops.op[q] == RED_MAX ? wave_max(a[q]) : wave_min(a[q]);
    if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    const int q = threadIdx.x;
    double x = red[q][0];
    for (int w = 1; w < W; ++w)
      x = ops.op[q] == RED_SUM ? x + red[q][w] : ops.op[q] == RED_MAX ? fmax(x, red[q][w]) : fmin(x, red[q][w]);
    out[q] = x;
  }
}

// ------------------------------------------------- mixed precision glue --
__global__ void __launch_bounds__(256)
k_set_f2d(double* __restrict__ db, double* __restrict__ dz, const float* __restrict__ eb,
          const float* __restrict__ ez, long long n) {
  CSIPM_ALIGN(db);
  CSIPM_ALIGN(dz);
  CSIPM_ALIGN(eb);
  CSIPM_ALIGN(ez);

  CSIPM_PAIRS(n) {
    db[i] = (double)eb[i];
    dz[i] = (double)ez[i];
  }
}

__global__ void __launch_bounds__(256)
k_add_f2d(double* __restrict__ db, double* __restrict__ dz, const float* __restrict__ eb,
          const float* __restrict__ ez, long long n) {
  CSIPM_ALIGN(db);
  CSIPM_ALIGN(dz);
  CSIPM_ALIGN(eb);
  CSIPM_ALIGN(ez);

  CSIPM_PAIRS(n) {
    db[i] += (double)eb[i];
    dz[i] += (double)ez[i];
  }
}

// FP32 start of a further inner solve of the refinement, elementwise from
// the residual pass's H d_beta: r = h - K d (FP64, K in Sigma form), r32 = r,
// z32 = p32 = P_c^{-1} r (formed in FP64), partial sums of r32.z32.
__global__ void __launch_bounds__(256)
k_ref_restart(const double* __restrict__ hb, const double* __restrict__ hz, const double* __restrict__ db,
              const double* __restrict__ dz, const double* __restrict__ hd, const double* __restrict__ s1,
              const double* __restrict__ s2, const float* __restrict__ c, float* __restrict__ frb,
              float* __restrict__ frz, float* __restrict__ fzb, float* __restrict__ fzz, float* __restrict__ fpb,
              float* __restrict__ fpz, long long n, double* partial) {
  CSIPM_ALIGN(hb);
  CSIPM_ALIGN(hz);
  CSIPM_ALIGN(db);
  CSIPM_ALIGN(dz);
  CSIPM_ALIGN(hd);
  CSIPM_ALIGN(s1);
  CSIPM_ALIGN(s2);
  CSIPM_ALIGN(frb);
  CSIPM_ALIGN(frz);
  CSIPM_ALIGN(fzb);
  CSIPM_ALIGN(fzz);
  CSIPM_ALIGN(fpb);
  CSIPM_ALIGN(fpz);

  double acc = 0.0;
  CSIPM_PAIRS(n) {
    double qb, qz, zb, zz;
    k_block<double>(hd[i], db[i], dz[i], s1[i], s2[i], qb, qz);
    const double rb = hb[i] - qb, rz = hz[i] - qz;
    pinv_block<double>(rb, rz, s1[i], s2[i], c ? (double)c[i] : 1.0, zb, zz);
    const float fb = (float)rb, fz = (float)rz, gb = (float)zb, gz = (float)zz;
    frb[i] = fb;
    frz[i] = fz;
    if (fzb) {
      fzb[i] = gb;
      fzz[i] = gz;
    }
    fpb[i] = gb;
    fpz[i] = gz;
    acc += (double)fb * (double)gb + (double)fz * (double)gz;
  }
  const int op = RED_SUM;
  block_reduce_store<1>(&acc, &op, partial, 0);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_pinv(const T* __restrict__ rb, const T* __restrict__ rz, T* __restrict__ zb, T* __restrict__ zz,
       const T* __restrict__ s1, const T* __restrict__ s2, const float* __restrict__ c, long long n,
       double* partial) {
  double acc = 0.0;
  for (long long i = gtid(); i < n; i += gstride()) {
    T ub, uz;
    pinv1<T>(rb[i], rz[i], s1[i], s2[i], c ? (double)c[i] : 1.0, ub, uz);
    zb[i] = ub;
    zz[i] = uz;
    acc += (double)rb[i] * (double)ub + (double)rz[i] * (double)uz;
  }
  const int op = RED_SUM;
  block_reduce_store<1>(&acc, &op, partial, 0);
}

// Non-finite count over observed samples of the signal.
__global__ void __launch_bounds__(256)
k_check_signal(const double* __restrict__ sig, const uint8_t* __restrict__ obs, long long n, double* partial) {
  double bad = 0.0, nobs = 0.0;
  for (long long i = gtid(); i < n; i += gstride()) {
    if (obs[i]) {
      nobs += 1.0;
      if (!isfinite(sig[i])) bad += 1.0;
    }
  }
  double v[2] = {bad, nobs};
  const int ops[2] = {RED_SUM, RED_SUM};
  block_reduce_store<2>(v, ops, partial, VEC_MAX_BLOCKS);
}

__global__ void __launch_bounds__(256)
k_zero_fill(const double* __restrict__ sig, const uint8_t* __restrict__ obs, double* __restrict__ out, long long n) {
  for (long long i = gtid(); i < n; i += gstride()) out[i] = obs[i] ? sig[i] : 0.0;
}

__global__ void __launch_bounds__(256)
k_obs_to_double(const uint8_t* __restrict__ obs, double* __restrict__ out, long long n) {
  for (long long i = gtid(); i < n; i += gstride()) out[i] = obs[i] ? 1.0 : 0.0;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_fill(T* __restrict__ a, T v, long long n) {
  for (long long i = gtid(); i < n; i += gstride()) a[i] = v;
}


__global__ void __launch_bounds__(256)
k_absmax(const double* __restrict__ a, long long n, double* partial) {
  double v = 0.0;
  for (long long i = gtid(); i < n; i += gstride()) v = fmax(v, fabs(a[i]));
  const int op = RED_MAX;
  block_reduce_store<1>(&v, &op, partial, 0);
}

// diag(M_perp^T M_perp) in the external beta layout from bm = A^T(mask):
// column i of A squared is (1/n)(1 + s_i cos(2 theta)), so
// H_ii = m/n + s_i Re(v_{2k}) / sqrt(n) with v the unitary DFT of the mask
// and s_i = +1 / -1 / 0 for the sqrt2 Re / sqrt2 Im / self-conjugate entry.
__global__ void __launch_bounds__(256)
k_diag_h(const double* __restrict__ bm, double* __restrict__ out, int n1, int n2, int n3, double mfrac,
         double rsqn) {
  const long long n = (long long)n1 * n2 * n3;
  const double rs2 = 0.70710678118654752440;
  for (long long f = gtid(); f < n; f += gstride()) {
    const int k3 = (int)(f % n3);
    const int k2 = (int)((f / n3) % n2);
    const int k1 = (int)(f / ((long long)n2 * n3));
    const int ck = cls3(k1, k2, k3, n1, n2, n3);
    const int q1 = (2 * k1) % n1, q2 = (2 * k2) % n2, q3 = (2 * k3) % n3;
    const int cq = cls3(q1, q2, q3, n1, n2, n3);
    double rev;
    if (cq == 0) {
      rev = bm[((long long)q1 * n2 + q2) * n3 + q3];
    } else if (cq == 1) {
      rev = rs2 * bm[((long long)q1 * n2 + q2) * n3 + q3];
    } else {
      const int m1 = (n1 - q1) % n1, m2 = (n2 - q2) % n2, m3 = (n3 - q3) % n3;
      rev = rs2 * bm[((long long)m1 * n2 + m2) * n3 + m3];
    }
    const double sgn = ck == 0 ? 0.0 : (ck == 1 ? 1.0 : -1.0);
    out[f] = mfrac + sgn * rev * rsqn;
  }
}

// Certificate sums of the LASSO solution beta (lasso_cert in vec.h); the
// natural residual uses g = -G: soft(beta + g, lam) = soft(beta - G, lam).
__global__ void __launch_bounds__(256)
k_lasso_cert(const double* __restrict__ beta, const double* __restrict__ g, double lam, long long n,
             double* partial) {
  double v[NCERT_Q] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long i = gtid(); i < n; i += gstride()) {
    const double b = beta[i], G = g[i];
    const double ab = fabs(b);
    v[0] += G * G;
    v[1] += ab;
    v[2] += lam * ab + b * G;
    v[3] += b * G;
    v[4] = fmax(v[4], fabs(G));
    const double x = b - G;
    const double sx = x > lam ? x - lam : (x < -lam ? x + lam : 0.0);
    v[5] = fmax(v[5], fabs(b - sx));
    v[6] = fmax(v[6], ab);
  }
  const int ops[NCERT_Q] = {RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_MAX, RED_MAX, RED_MAX};
  block_reduce_store<NCERT_Q>(v, ops, partial, VEC_MAX_BLOCKS);
}

}  // namespace

int vec_blocks(long long n) {
  long long b = (n + 1023) / 1024;
  if (b > VEC_MAX_BLOCKS) b = VEC_MAX_BLOCKS;
  if (b < 1) b = 1;
  return (int)b;
}

#define VB dim3(vec_blocks(n)), dim3(256), 0, s

template <typename T>
void cg_update(T* xb, T* xz, const T* pb, const T* pz, const T* qb, const T* qz, T* rb, T* rz, T* zb, T* zz,
               const T* s1, const T* s2, const float* c, const double* scal, const int* flags, long long n,
               double* partial, bool first, hipStream_t s) {
  hipLaunchKernelGGL((k_cg_update<T>), VB, xb, xz, pb, pz, qb, qz, rb, rz, zb, zz, s1, s2, c, scal, flags, n,
                     partial, first ? 1 : 0);
}
void fin_cg_start(const double* partial, int nb, int stride, double* scal, int* flags, double eta, double atol,
                  int maxit, int ref_slot, int from_slot, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_cg_init, dim3(1), dim3(256), 0, s, partial, nb, stride, scal, flags, eta, atol, maxit,
                     ref_slot, from_slot);
}
template <typename TC>
void newton_init(const double* beta, const double* z, const double* nu1, const double* nu2, const double* hb,
                 double lam, double smu, double* sig1, double* sig2, double* hb_out,
                 double* hz_out, TC* sig1c, TC* sig2c, const float* c, TC* rb, TC* rz, TC* zb, TC* zz, TC* pb,
                 TC* pz, long long n, double* partial, hipStream_t s, const double* dab, const double* daz) {
  if (dab)   // corrector of a predictor-corrector step
    hipLaunchKernelGGL((k_newton_init<TC, true>), VB, beta, z, nu1, nu2, hb, lam, smu, sig1, sig2, hb_out, hz_out,
                       sig1c, sig2c, c, rb, rz, zb, zz, pb, pz, n, partial, dab, daz);
  else
    hipLaunchKernelGGL((k_newton_init<TC, false>), VB, beta, z, nu1, nu2, hb, lam, smu, sig1, sig2, hb_out, hz_out,
                       sig1c, sig2c, c, rb, rz, zb, zz, pb, pz, n, partial, dab, daz);
}
void set_f2d(double* db, double* dz, const float* eb, const float* ez, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_set_f2d, VB, db, dz, eb, ez, n);
}
void fin_alpha(const double* partial, int nb, double* scal, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(256), 0, s, partial, nb, scal, flags);
}
template <typename T>
void cr_dir(T* pb, T* pz, T* qb, T* qz, const T* zb, const T* zz, const T* wb, const T* wz, const T* s1, const T* s2,
            const float* c, const double* scal, const int* flags, long long n, double* partial, bool first,
            hipStream_t s) {
  hipLaunchKernelGGL((k_cr_dir<T>), VB, pb, pz, qb, qz, zb, zz, wb, wz, s1, s2, c, scal, flags, n, partial,
                     first ? 1 : 0);
}
template <typename T>
void car_dir(T* pb, T* pz, T* vb, T* vz, T* yb, T* yz, const T* zb, const T* zz, const T* ub, const T* uz,
             const T* sb, const T* sz, const T* s1, const T* s2, const float* c, const double* scal,
             const int* flags, long long n, double* partial, bool first, hipStream_t s) {
  hipLaunchKernelGGL((k_car_dir<T>), VB, pb, pz, vb, vz, yb, yz, zb, zz, ub, uz, sb, sz, s1, s2, c, scal, flags, n,
                     partial, first ? 1 : 0);
}
template <typename T>
void car_update(T* xb, T* xz, const T* pb, const T* pz, T* zb, T* zz, const T* vb, const T* vz, T* ub, T* uz,
                const T* yb, const T* yz, const T* s1, const T* s2, const float* c, const double* scal,
                const int* flags, long long n, double* partial, bool first, hipStream_t s) {
  hipLaunchKernelGGL((k_car_update<T>), VB, xb, xz, pb, pz, zb, zz, vb, vz, ub, uz, yb, yz, s1, s2, c, scal, flags,
                     n, partial, first ? 1 : 0);
}
template <typename T>
void p_apply(const T* zb, const T* zz, const T* s1, const T* s2, const float* c, T* rb, T* rz, long long n,
             hipStream_t s) {
  hipLaunchKernelGGL((k_p_apply<T>), VB, zb, zz, s1, s2, c, rb, rz, n);
}
void fin_cr_zw(const double* partial, int nb, double* scal, int* flags, bool first, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_cr_zw, dim3(1), dim3(256), 0, s, partial, nb, scal, flags, first ? 1 : 0);
}
void fin_rz(const double* partial, int nb, double* scal, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_rz, dim3(1), dim3(256), 0, s, partial, nb, scal, flags);
}
void ipm_init(double* beta, double* z, double* nu1, double* nu2, double* g, const double* xi, long long n, double z0,
              double lam, hipStream_t s) {
  hipLaunchKernelGGL(k_ipm_init, VB, beta, z, nu1, nu2, g, xi, n, z0, lam);
}
static const RedOps<NRESID> kResidRedOps{CSIPM_RESID_OPS};

void ipm_resid(const double* beta, const double* z, const double* nu1, const double* nu2, double* hb,
               const double* xi, double lam, long long n, double* partial, double* out8, bool logsum, hipStream_t s) {
  const int nb = vec_blocks(n);
  hipLaunchKernelGGL(k_ipm_resid, VB, beta, z, nu1, nu2, hb, xi, lam, n, partial, VEC_MAX_BLOCKS, logsum ? 1 : 0);
  hipLaunchKernelGGL((k_fin_reduce<NRESID>), dim3(1), dim3(kFinThreads), 0, s, partial, nb, VEC_MAX_BLOCKS, out8,
                     kResidRedOps);
}
void ipm_step(const double* beta, const double* z, const double* nu1, const double* nu2, const double* db,
              const double* dz, const float* db32, const float* dz32, double smu, double tau, long long n,
              double* partial, double* scal, hipStream_t s, const double* dab, const double* daz, double* dsdn,
              bool next_smu, double s0, double sigma) {
  const int nb = vec_blocks(n);
  const bool d32 = db32 != nullptr, corr = dab != nullptr;
#define CSIPM_RATIO(B, C, D)                                                                                     \
  do {                                                                                                           \
    if (d32)                                                                                                     \
      hipLaunchKernelGGL((k_ipm_ratio<true, B, C, D>), VB, beta, z, nu1, nu2, db, dz, db32, dz32, smu, n, partial, \
                         dab, daz);                                                                              \
    else                                                                                                         \
      hipLaunchKernelGGL((k_ipm_ratio<false, B, C, D>), VB, beta, z, nu1, nu2, db, dz, db32, dz32, smu, n,        \
                         partial, dab, daz);                                                                     \
  } while (0)
  if (next_smu)   // (standard steps only)
    CSIPM_RATIO(false, false, true);
  else if (dsdn)  // (the affine direction of a predictor-corrector step)
    CSIPM_RATIO(false, true, false);
  else if (corr)
    CSIPM_RATIO(true, false, false);
  else
    CSIPM_RATIO(false, false, false);
#undef CSIPM_RATIO
  hipLaunchKernelGGL(k_fin_step, dim3(1), dim3(256), 0, s, partial, nb, tau, scal, next_smu ? 1 : 0, s0, sigma,
                     0.5 / (double)n);
  if (dsdn) {
    RedOps<1> ops{{RED_SUM}};
    hipLaunchKernelGGL((k_fin_reduce<1>), dim3(1), dim3(kFinThreads), 0, s, partial + VEC_MAX_BLOCKS, nb, VEC_MAX_BLOCKS,
                       dsdn, ops);
  }
}
void ipm_advance(double* beta, double* z, double* nu1, double* nu2, double* hbeta, const double* db, const double* dz,
                 const float* db32, const float* dz32, const double* hd, const double* rres, const float* rres32,
                 double lam, double smu, double* scal, long long n, double* partial, bool logsum, hipStream_t s,
                 const double* dab, const double* daz, const NextSystem* next, uint32_t* act) {
  const int nb = vec_blocks(n);
  const int hdm = hd ? ADV_DIRECT : rres32 ? ADV_RRES32 : ADV_RRES64;
  // (an FP32 direction comes only with the FP32 residual)
  const int ls = logsum ? 1 : 0;
#define CSIPM_ADV(TC, NI, HDM, CORR, NO, CN)                                                                        \
  hipLaunchKernelGGL((k_ipm_advance<TC, NI, HDM, CORR>), VB, beta, z, nu1, nu2, hbeta, db, dz, hd, rres, rres32,    \
                     db32, dz32, lam, smu, scal, n, partial, VEC_MAX_BLOCKS, ls, dab, daz, NO, CN, act)
  if (next && next->out32) {   // (standard steps: no corrector terms)
    if (hdm == ADV_DIRECT)
      CSIPM_ADV(float, true, ADV_DIRECT, false, *next->out32, next->c);
    else
      CSIPM_ADV(float, true, ADV_RRES32, false, *next->out32, next->c);
  } else if (next && next->out64) {
    CSIPM_ADV(double, true, ADV_RRES64, false, *next->out64, next->c);
  } else if (dab) {
    if (hdm == ADV_DIRECT)
      CSIPM_ADV(float, false, ADV_DIRECT, true, NewtonOut<float>{}, nullptr);
    else if (hdm == ADV_RRES32)
      CSIPM_ADV(float, false, ADV_RRES32, true, NewtonOut<float>{}, nullptr);
    else
      CSIPM_ADV(float, false, ADV_RRES64, true, NewtonOut<float>{}, nullptr);
  } else {
    if (hdm == ADV_DIRECT)
      CSIPM_ADV(float, false, ADV_DIRECT, false, NewtonOut<float>{}, nullptr);
    else if (hdm == ADV_RRES32)
      CSIPM_ADV(float, false, ADV_RRES32, false, NewtonOut<float>{}, nullptr);
    else
      CSIPM_ADV(float, false, ADV_RRES64, false, NewtonOut<float>{}, nullptr);
  }
#undef CSIPM_ADV
  hipLaunchKernelGGL((k_fin_reduce<NRESID>), dim3(1), dim3(kFinThreads), 0, s, partial, nb, VEC_MAX_BLOCKS, scal + S_RESID,
                     kResidRedOps);
}
void add_f2d(double* db, double* dz, const float* eb, const float* ez, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_add_f2d, VB, db, dz, eb, ez, n);
}
void ref_restart(const double* hb, const double* hz, const double* db, const double* dz, const double* hd,
                 const double* s1, const double* s2, const float* c, float* frb, float* frz, float* fzb, float* fzz,
                 float* fpb, float* fpz, long long n, double* partial, double* out, hipStream_t s) {
  const int nb = vec_blocks(n);
  hipLaunchKernelGGL(k_ref_restart, VB, hb, hz, db, dz, hd, s1, s2, c, frb, frz, fzb, fzz, fpb, fpz, n, partial);
  fin_sum(partial, nb, out, s);
}
void fin_sum(const double* partial, int nb, double* out, hipStream_t s) {
  RedOps<1> ops{{RED_SUM}};
  hipLaunchKernelGGL((k_fin_reduce<1>), dim3(1), dim3(kFinThreads), 0, s, partial, nb, VEC_MAX_BLOCKS, out, ops);
}
void fin_max(const double* partial, int nb, double* out, hipStream_t s) {
  RedOps<1> ops{{RED_MAX}};
  hipLaunchKernelGGL((k_fin_reduce<1>), dim3(1), dim3(kFinThreads), 0, s, partial, nb, VEC_MAX_BLOCKS, out, ops);
}
template <typename T>
void pinv_apply(const T* rb, const T* rz, T* zb, T* zz, const T* s1, const T* s2, const float* c, long long n,
                double* partial, double* out, hipStream_t s) {
  const int nb = vec_blocks(n);
  hipLaunchKernelGGL((k_pinv<T>), VB, rb, rz, zb, zz, s1, s2, c, n, partial);
  if (out) {
    RedOps<1> ops{{RED_SUM}};
    hipLaunchKernelGGL((k_fin_reduce<1>), dim3(1), dim3(kFinThreads), 0, s, partial, nb, VEC_MAX_BLOCKS, out,
                       ops);
  }
}
void check_signal(const double* sig, const uint8_t* obs, long long n, double* partial, double* out2, hipStream_t s) {
  const int nb = vec_blocks(n);
  hipLaunchKernelGGL(k_check_signal, VB, sig, obs, n, partial);
  RedOps<2> ops{{RED_SUM, RED_SUM}};
  hipLaunchKernelGGL((k_fin_reduce<2>), dim3(1), dim3(kFinThreads), 0, s, partial, nb, VEC_MAX_BLOCKS, out2, ops);
}
void zero_fill(const double* sig, const uint8_t* obs, double* out, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_fill, VB, sig, obs, out, n);
}
void obs_to_double(const uint8_t* obs, double* out, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_obs_to_double, VB, obs, out, n);
}
template <typename T>
void fill(T* a, T v, long long n, hipStream_t s) {
  hipLaunchKernelGGL((k_fill<T>), VB, a, v, n);
}
void absmax(const double* a, long long n, double* partial, double* out, hipStream_t s) {
  const int nb = vec_blocks(n);
  hipLaunchKernelGGL(k_absmax, VB, a, n, partial);
  RedOps<1> ops{{RED_MAX}};
  hipLaunchKernelGGL((k_fin_reduce<1>), dim3(1), dim3(kFinThreads), 0, s, partial, nb, VEC_MAX_BLOCKS, out, ops);
}
void lasso_cert(const double* beta, const double* g, double lam, long long n, double* partial, double* out,
                hipStream_t s) {
  const int nb = vec_blocks(n);
  hipLaunchKernelGGL(k_lasso_cert, VB, beta, g, lam, n, partial);
  RedOps<NCERT_Q> ops{{RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_MAX, RED_MAX, RED_MAX}};
  hipLaunchKernelGGL((k_fin_reduce<NCERT_Q>), dim3(1), dim3(kFinThreads), 0, s, partial, nb, VEC_MAX_BLOCKS, out,
                     ops);
}
void diag_h(const double* bm_ext, double* out_ext, int n1, int n2, int n3, double mfrac, hipStream_t s) {
  const long long n = (long long)n1 * n2 * n3;
  hipLaunchKernelGGL(k_diag_h, VB, bm_ext, out_ext, n1, n2, n3, mfrac, 1.0 / std::sqrt((double)n));
}

#undef VB

#define CSIPM_VINST(T)                                                                                         \
  template void cg_update<T>(T*, T*, const T*, const T*, const T*, const T*, T*, T*, T*, T*, const T*,         \
                             const T*, const float*, const double*, const int*, long long, double*, bool,      \
                             hipStream_t);                                                                     \
  template void newton_init<T>(const double*, const double*, const double*, const double*, const double*,     \
                               double, double, double*, double*, double*, double*, T*, T*,                     \
                               const float*, T*, T*, T*, T*, T*, T*, long long, double*, hipStream_t,          \
                               const double*, const double*);                                                  \
  template void cr_dir<T>(T*, T*, T*, T*, const T*, const T*, const T*, const T*, const T*, const T*,         \
                          const float*, const double*, const int*, long long, double*, bool, hipStream_t);   \
  template void car_dir<T>(T*, T*, T*, T*, T*, T*, const T*, const T*, const T*, const T*, const T*, const T*,  \
                           const T*, const T*, const float*, const double*, const int*, long long, double*,    \
                           bool, hipStream_t);                                                                 \
  template void car_update<T>(T*, T*, const T*, const T*, T*, T*, const T*, const T*, T*, T*, const T*,      \
                              const T*, const T*, const T*, const float*, const double*, const int*, long long, \
                              double*, bool, hipStream_t);                                                     \
  template void p_apply<T>(const T*, const T*, const T*, const T*, const float*, T*, T*, long long,           \
                           hipStream_t);                                                                       \
  template void pinv_apply<T>(const T*, const T*, T*, T*, const T*, const T*, const float*, long long,        \
                              double*, double*, hipStream_t);                                                  \
  template void fill<T>(T*, T, long long, hipStream_t);
CSIPM_VINST(double)
CSIPM_VINST(float)
#undef CSIPM_VINST

}  // namespace csipm
