// Learned diagonal correction of the preconditioner: kernel launchers.
//
// Network 4 -> 32 -> 32 -> 1 with tanh hidden units and c = softplus(o)+1e-6,
// float32 parameters in the flat layout W1[32][4], b1[32], W2[32][32], b2[32],
// w3[32], b3 (1249 values).  Features per coefficient i:
//   f1 = log L1_i - mean log L1,  f2 = L2_i / L1_i,
//   f3 = log(|beta_i| / max|beta| + 1e-12),  f4 = diag(M_perp^T M_perp)_i.
// Training record of a sampled coefficient i of a Krylov direction p with
// u = H p_beta: {u_i, p_beta_i, L1_i, L2_i, 4 S1_i S2_i, w_i}; its loss is
//   w (L1^2 + L2^2)(u - c p)^2 / (L1 + 4 S1 S2)^2,
// the squared i-th block of P^{-1}(K - P_c)p with P the paper's
// preconditioner: a weighted least-squares fit of c_i p_i to (H p)_i.
#pragma once

#include "csipm_internal.h"

namespace csipm {

constexpr int MLP_NP = 1249;
constexpr int MLP_REC = 6;
constexpr int MLP_REC_PER_BLOCK = 64;   // records per training workgroup (one gradient partial each)

// mean of log(S1 + S2) over n coefficients -> *out (device), via partials
void mlp_mean_log_l1(const double* s1, const double* s2, long long n, double* partial, double* out, hipStream_t s);
// feat[i][4] from the iterate (internal order); meanlog and bmax are device scalars
void mlp_features(const double* s1, const double* s2, const double* beta, const double* diagH,
                  const double* meanlog, const double* bmax, float* feat, long long n, hipStream_t s);
// features of the interior-point state (Sigma formed from beta, z, nu)
void mlp_features_state(const double* beta, const double* z, const double* nu1, const double* nu2,
                        const double* diagH, const double* bmax, float* feat, long long n, double* partial,
                        double* meanlog, hipStream_t s);
// mean of log(S1 + S2) of the interior-point state -> *meanlog (device)
void mlp_mean_log_l1_state(const double* beta, const double* z, const double* nu1, const double* nu2, long long n,
                           double* partial, double* meanlog, hipStream_t s);
// c of the interior-point state, network evaluated (on the matrix cores) only
// where pc_gate passes (c = 1 elsewhere); the centring of the first feature
// is *meanlog * mscale, and meanlog, bmax are device scalars; set[k] = 1 for
// the 64-coefficient chunks k where c may differ from 1, else 0
void mlp_correction_state(const double* beta, const double* z, const double* nu1, const double* nu2,
                          const double* diagH, const double* meanlog, double mscale, const double* bmax,
                          const float* params, float* c, long long n, uint32_t* set, hipStream_t s);
// c of the interior-point state as mlp_correction_state forms it, for an
// iterate whose Newton system (Sigma s1c/s2c, r = rb/rz, p = pb/pz in TC;
// for TC = float also the FP64 Sigma s164/s264 and h hb64/hz64, or null)
// was built with c = 1 and whose chunks the update flagged in act: p is
// rewritten to P_c^{-1} r where c acts, and the change of r.P^{-1}r (and
// h.P^{-1}h) is added to partial[b] (and partial[stride + b]) for workgroup
// b < max_blocks.  Only flagged chunks and those set marks are visited
// (with tracked false, every chunk: c may then differ from 1 anywhere);
// set is updated.
template <typename TC>
void mlp_correction_patch(const double* beta, const double* z, const double* nu1, const double* nu2,
                          const double* diagH, const double* meanlog, double mscale, const double* bmax,
                          const float* params, float* c, long long n, const uint32_t* act, uint32_t* set,
                          bool tracked, const TC* s1c, const TC* s2c, const TC* rb, const TC* rz, TC* pb, TC* pz,
                          const double* s164, const double* s264, const double* hb64, const double* hz64,
                          double* partial, int stride, int max_blocks, hipStream_t s);
// c = softplus(MLP(feat)) + 1e-6 for n records (matrix-core inference)
void mlp_forward(const float* params, const float* feat, float* c, long long n, hipStream_t s);
// gradient of sum_i dc_i c_i, accumulated into grad (float, 1249)
void mlp_backward(const float* params, const float* feat, const float* dc, float* grad, int n, double* scratch,
                  hipStream_t s);
// loss (double, device) and gradient (float, overwritten) over n records;
// scratch holds ceil(n/128) * 1250 doubles
void mlp_loss_grad(const float* params, const float* feat, const float* rec, int n, double* loss, float* grad,
                   double* scratch, hipStream_t s);
void mlp_adam(float* params, const float* grad, float* m, float* v, int t, float lr, hipStream_t s);

// Capture: records at coefficients idx_j = splitmix64(seed + j) mod n,
// j < npick, from (p, q = K p) and the barrier diagonals; feat_all is the
// full [n][4] feature array of the iterate.  w_j = 1 / sum_j (pb^2 + pz^2).
// With gate_idx (n ints of scratch) the coefficients are drawn only among
// those where L1 / (L1 + 4 S1 S2) >= rmin; partial must then hold
// 8192 + 1024 doubles.
template <typename T>
void mlp_capture(const T* pb, const T* pz, const T* qb, const T* qz, const T* s1, const T* s2,
                 const float* feat_all, long long n, int npick, unsigned long long seed, float* out_feat,
                 float* out_rec, double* partial, int* gate_idx, double rmin, hipStream_t s);
void mlp_scale_weights(float* rec, int npick, float factor, hipStream_t s);

}  // namespace csipm
