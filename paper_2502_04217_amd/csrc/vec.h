// Krylov / interior-point kernel launchers (vec.hip) and the device scalar
// slots they share with the host driver.
#pragma once

#include "csipm_internal.h"

namespace csipm {

constexpr int VEC_MAX_BLOCKS = 2048;   // partial sums per reduced quantity

enum RedOp { RED_SUM = 0, RED_MAX = 1, RED_MIN = 2 };
template <int NQ>
struct RedOps {
  int op[NQ];
};

// double slots of the device scalar block
enum ScalarSlot {
  S_RZ = 0,        // current r.P^{-1}r
  S_RZ0 = 1,       // initial r.P^{-1}r
  S_PQ = 2,        // p.Kp
  S_ALPHA = 3,     // CG step
  S_BETA = 4,      // CG direction update
  S_TOL = 5,       // stopping threshold on sqrt(r.P^{-1}r)
  S_RES = 6,       // sqrt(r.P^{-1}r) now
  S_ZW = 7,        // conjugate residuals: z.K z of the current iterate
  S_AMAX = 8,      // IPM: largest feasible step
  S_ALPHA_IPM = 9, // IPM: step taken
  S_REF = 10,      // refinement: r.P^{-1}r of the FP64 residual
  S_REF0 = 11,     // refinement: rhs.P^{-1}rhs
  S_REFRZ = 12,    // refinement: r32.P^{-1}r32, start of the next inner PCG
  S_REFINF = 13,   // refinement: max |r| of the FP64 residual
  S_DSDN = 14,     // predictor-corrector: sum ds.dnu of the affine direction
  S_SMU = 15,      // target sigma mu of the next Newton system built with the step
  S_RESID = 16,    // IPM residual block, 10 values (k_ipm_resid order)
  S_SIG = 28,      // signal check: non-finite count, observed count
  S_MISC = 32,     // free scratch (8 values)
  S_CERT = 40,     // LASSO certificate sums of lasso_cert (NCERT_Q values)
  S_COUNT = 64
};
// int slots of the device flag block
enum FlagSlot { F_DONE = 0, F_IT = 1, F_MAXIT = 2, F_BREAK = 3, F_COUNT = 8 };

int vec_blocks(long long n);

template <typename T>
void cg_update(T* xb, T* xz, const T* pb, const T* pz, const T* qb, const T* qz, T* rb, T* rz, T* zb, T* zz,
               const T* s1, const T* s2, const float* c, const double* scal, const int* flags, long long n,
               double* partial, bool first, hipStream_t s);
// conjugate residuals: p = z + beta p, q = w + beta q (p = z, q = w first),
// partial q.P_c^{-1}q; and the finalize after w = K z (beta, alpha's numerator)
template <typename T>
void cr_dir(T* pb, T* pz, T* qb, T* qz, const T* zb, const T* zz, const T* wb, const T* wz, const T* s1, const T* s2,
            const float* c, const double* scal, const int* flags, long long n, double* partial, bool first,
            hipStream_t s);
void fin_cr_zw(const double* partial, int nb, double* scal, int* flags, bool first, hipStream_t s);
// r = P_c z (elementwise 2x2 blocks)
template <typename T>
void p_apply(const T* zb, const T* zz, const T* s1, const T* s2, const float* c, T* rb, T* rz, long long n,
             hipStream_t s);
// conjugate A-residuals: direction step (p, v = P^{-1}Kp, y = P^{-1}Kv from
// s = K u; partial y.P y) and update (x, z = P^{-1}r, u = P^{-1}Kz; partial
// z.P z)
template <typename T>
void car_dir(T* pb, T* pz, T* vb, T* vz, T* yb, T* yz, const T* zb, const T* zz, const T* ub, const T* uz,
             const T* sb, const T* sz, const T* s1, const T* s2, const float* c, const double* scal,
             const int* flags, long long n, double* partial, bool first, hipStream_t s);
template <typename T>
void car_update(T* xb, T* xz, const T* pb, const T* pz, T* zb, T* zz, const T* vb, const T* vz, T* ub, T* uz,
                const T* yb, const T* yz, const T* s1, const T* s2, const float* c, const double* scal,
                const int* flags, long long n, double* partial, bool first, hipStream_t s);
// rz0 from partial quantity 0 (or scal[from_slot] when >= 0); quantity 1
// (at partial + stride) summed into scal[ref_slot] when ref_slot >= 0
void fin_cg_start(const double* partial, int nb, int stride, double* scal, int* flags, double eta, double atol,
                  int maxit, int ref_slot, int from_slot, hipStream_t s);
// The interior-point iteration carries G = H beta - xi (the "hb" arrays
// below), the data part of the first KKT residual row.
//
// Newton system of the iterate: Sigma, h, r = h and p = z = P_c^{-1} r (z
// skipped when zb is null: CG never reads it before its first update), the
// sums r.z and h.P^{-1}h
// Where a Newton system build writes: FP64 Sigma and h (each pair nullable),
// Sigma in the Krylov precision TC (FP32 only), r = h, z = P_c^{-1} r (zb
// nullable) and p = z.
template <typename TC>
struct NewtonOut {
  double *sig1, *sig2, *hb_out, *hz_out;
  TC *sig1c, *sig2c, *rb, *rz, *zb, *zz, *pb, *pz;
};
// the next Newton system built by ipm_advance: in FP32 (out32) or FP64
// (out64) Krylov precision, with correction c (null: none)
struct NextSystem {
  const NewtonOut<float>* out32;
  const NewtonOut<double>* out64;
  const float* c;
};
// quantities reduced by ipm_advance (its partials of the next system follow)
constexpr int NRESID_Q = 10;

template <typename TC>
void newton_init(const double* beta, const double* z, const double* nu1, const double* nu2, const double* hb,
                 double lam, double smu, double* sig1, double* sig2, double* hb_out,
                 double* hz_out, TC* sig1c, TC* sig2c, const float* c, TC* rb, TC* rz, TC* zb, TC* zz, TC* pb,
                 TC* pz, long long n, double* partial, hipStream_t s, const double* dab = nullptr,
                 const double* daz = nullptr);
void set_f2d(double* db, double* dz, const float* eb, const float* ez, long long n, hipStream_t s);
void fin_alpha(const double* partial, int nb, double* scal, int* flags, hipStream_t s);
void fin_rz(const double* partial, int nb, double* scal, int* flags, hipStream_t s);

// beta = 0, z = z0, nu = lam/2, and G = -xi (H beta = 0)
void ipm_init(double* beta, double* z, double* nu1, double* nu2, double* g, const double* xi, long long n, double z0,
              double lam, hipStream_t s);
// residual parts of the iterate -> out8 (k_ipm_resid order; out8[7] = sum
// log(S1 + S2) when logsum).  hb holds G, or H beta when xi is set, which is
// then replaced in place by G = H beta - xi.
void ipm_resid(const double* beta, const double* z, const double* nu1, const double* nu2, double* hb,
               const double* xi, double lam, long long n, double* partial, double* out8, bool logsum, hipStream_t s);
// step length: scal[S_AMAX] and scal[S_ALPHA_IPM] = min(1, tau * S_AMAX)
// (the direction is read from db32/dz32 when set, else from db/dz)
// (dab, daz: the affine direction of a predictor-corrector step, for the
// corrector's dnu; dsdn: where to put sum ds.dnu of this direction)
// (next_smu: also scal[S_SMU] = sigma mu+, mu+ the duality measure after the
// step from s0 = sum s.nu now and the sums of the ratio pass)
void ipm_step(const double* beta, const double* z, const double* nu1, const double* nu2, const double* db,
              const double* dz, const float* db32, const float* dz32, double smu, double tau, long long n,
              double* partial, double* scal, hipStream_t s, const double* dab = nullptr, const double* daz = nullptr,
              double* dsdn = nullptr, bool next_smu = false, double s0 = 0.0, double sigma = 0.0);
// iterate update with G carried along (H d_beta from hd when set, else
// from the Krylov residual: rres32 when set, else rres), and the new residual
// parts -> scal[S_RESID..]; with rres, scal[S_RESID + 9] = max (S1 + S2)
// (|d_beta| + |d_z|), which times the FP64 epsilon bounds the rounding error
// of the recovered H d_beta
// (next: also build the next Newton system from the new iterate at target
// scal[S_SMU], as newton_init would with correction next->c; its r.z and
// h.P^{-1}h partials stay in quantities NRESID_Q and NRESID_Q + 1 of partial)
// (act: also act[c] = 1 where chunk c (coefficients 64c .. 64c + 63) of the
// new iterate holds one where the correction's gate passes, else 0; the
// launch covers n / 2 pairs in waves of 64 consecutive pairs)
void ipm_advance(double* beta, double* z, double* nu1, double* nu2, double* hbeta, const double* db,
                 const double* dz, const float* db32, const float* dz32, const double* hd,
                 const double* rres, const float* rres32, double lam, double smu, double* scal, long long n,
                 double* partial, bool logsum, hipStream_t s, const double* dab = nullptr,
                 const double* daz = nullptr, const NextSystem* next = nullptr, uint32_t* act = nullptr);

void add_f2d(double* db, double* dz, const float* eb, const float* ez, long long n, hipStream_t s);
// FP32 restart of a further inner solve from H d_beta (hd): r32, z32 = p32 =
// P_c^{-1} r (z32 skipped when fzb is null) and the sum r32.z32 -> *out
// (device)
void ref_restart(const double* hb, const double* hz, const double* db, const double* dz, const double* hd,
                 const double* s1, const double* s2, const float* c, float* frb, float* frz, float* fzb, float* fzz,
                 float* fpb, float* fpz, long long n, double* partial, double* out, hipStream_t s);
// *out = sum of partial[0..nb)
void fin_sum(const double* partial, int nb, double* out, hipStream_t s);
// *out = max of partial[0..nb)
void fin_max(const double* partial, int nb, double* out, hipStream_t s);
template <typename T>
void pinv_apply(const T* rb, const T* rz, T* zb, T* zz, const T* s1, const T* s2, const float* c, long long n,
                double* partial, double* out, hipStream_t s);
void check_signal(const double* sig, const uint8_t* obs, long long n, double* partial, double* out2, hipStream_t s);
void zero_fill(const double* sig, const uint8_t* obs, double* out, long long n, hipStream_t s);
void obs_to_double(const uint8_t* obs, double* out, long long n, hipStream_t s);
template <typename T>
void fill(T* a, T v, long long n, hipStream_t s);
void absmax(const double* a, long long n, double* partial, double* out, hipStream_t s);
void diag_h(const double* bm_ext, double* out_ext, int n1, int n2, int n3, double mfrac, hipStream_t s);

// LASSO optimality and duality gap of beta (equation "realopt" and its dual)
// from G = H beta - xi = -M_perp^T r, r = b - M_perp beta (M_perp^T is an
// isometry on the observed samples, so ||r|| = ||G||).  out[0..NCERT_Q):
//   sum G^2 (= ||r||^2), sum |beta|, sum (lam |beta_i| + beta_i G_i)
//   (= lam ||beta||_1 - beta.g, summed termwise), sum beta_i G_i,
//   max |G| (= ||g||_inf), max |beta - soft(beta - G, lam)|, max |beta|
constexpr int NCERT_Q = 7;
void lasso_cert(const double* beta, const double* g, double lam, long long n, double* partial, double* out,
                hipStream_t s);

}  // namespace csipm
