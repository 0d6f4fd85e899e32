// Learned diagonal correction of the preconditioner: feature, inference,
// training (forward + backward + Adam) and record-capture kernels.  Not in
// the paper, whose preconditioner P = [[I + L1, L2], [L2, L1]] this corrects
// (I -> diag(c), c > 0 keeps every 2x2 block positive definite).
#include "mlp.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace csipm {

namespace {

constexpr int H1 = 32, H2 = 32, NIN = 4;
constexpr int OW1 = 0, OB1 = OW1 + H1 * NIN, OW2 = OB1 + H1, OB2 = OW2 + H2 * H1, OW3 = OB2 + H2, OB3 = OW3 + H2;
static_assert(OB3 + 1 == MLP_NP, "parameter layout");
constexpr int RB = MLP_REC_PER_BLOCK;   // records per training workgroup
constexpr int RP = RB + 1;      // padded LDS row
constexpr int kGateBlocks = 1024;   // workgroups listing the coefficients where the correction acts

__device__ __forceinline__ long long gtid() { return blockIdx.x * (long long)blockDim.x + threadIdx.x; }
__device__ __forceinline__ long long gstride() { return (long long)gridDim.x * blockDim.x; }


// tanh in float32 to ~2e-7 relative: an odd polynomial (least-squares fit
// of tanh(x)/x in x^2 on [0, 0.55]) below 0.55, 1 - 2/(exp(2|x|) + 1) above.
__device__ __forceinline__ float tanh_fast(float x) {
  const float ax = fabsf(x);
  if (ax < 0.55f) {
    const float t = x * x;
    float p = -0.0063321318888434315f;
    p = fmaf(p, t, 0.021107190038856506f);
    p = fmaf(p, t, -0.05385906545947602f);
    p = fmaf(p, t, 0.13332620512105214f);
    p = fmaf(p, t, -0.33333316330560286f);
    p = fmaf(p, t, 0.9999999993472424f);
    return x * p;
  }
  const float e = __expf(2.0f * ax);
  return copysignf(1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f), x);
}
__device__ __forceinline__ float softplusf(float x) { return fmaxf(x, 0.0f) + log1pf(__expf(-fabsf(x))); }
__device__ __forceinline__ float sigmoidf(float x) { return 0.5f * (1.0f + tanh_fast(0.5f * x)); }

__device__ __forceinline__ void load_params(const float* __restrict__ g, float* s) {
  for (int i = threadIdx.x; i < MLP_NP; i += blockDim.x) s[i] = g[i];
  __syncthreads();
}

// forward of one coefficient; returns o (pre-activation of the output)
__device__ __forceinline__ float fwd1(const float* P, const float x[NIN], float h1[H1], float h2[H2]) {
#pragma unroll
  for (int i = 0; i < H1; ++i) {
    float a = P[OB1 + i];
#pragma unroll
    for (int j = 0; j < NIN; ++j) a = fmaf(P[OW1 + i * NIN + j], x[j], a);
    h1[i] = tanh_fast(a);
  }
  float o = P[OB3];
#pragma unroll 4
  for (int i = 0; i < H2; ++i) {
    float a = P[OB2 + i];
#pragma unroll
    for (int j = 0; j < H1; ++j) a = fmaf(P[OW2 + i * H1 + j], h1[j], a);
    h2[i] = tanh_fast(a);
    o = fmaf(P[OW3 + i], h2[i], o);
  }
  return o;
}

// ------------------------------------------------ inference on MFMA --
// Inference runs the two dense layers on the matrix cores
// (v_mfma_f32_16x16x4_f32, FP32 in, FP32 accumulate) with coefficients along
// the 16 columns and neurons along the rows.  Register layout of that MFMA
// for lane l (g = l / 16, q = l % 16): A is 16x4 with lane l holding A[q][g],
// B is 4x16 with lane l holding B[g][q], D is 16x16 with lane l holding
// D[4g + r][q] in register r.  Layer 1 (K = 4 features) is one MFMA per 16
// neurons.  A layer output lands in lane (g, q) as neurons 16t + 4g + r of
// coefficient q, which is already a valid B operand for the next layer if the
// contraction index of k-step (t, r) is taken as g <-> neuron 16t + 4g + r;
// the A operand (weights) is permuted to match, so no data moves between
// layers.
typedef float f4_t __attribute__((ext_vector_type(4)));

struct MfmaNet {
  float w1[2];      // W1[16t + q][g]
  float w2[2][8];   // output rows 16m + q, k-step s = 4t + r: W2[16m + q][16t + 4g + r]
  float b1[2][4];   // [t][r]: b1[16t + 4g + r]
  float b2[2][4];
  float w3[2][4];
  float b3;
};

__device__ __forceinline__ void load_net(const float* __restrict__ P, MfmaNet& w) {
  const int l = threadIdx.x & 63, g = l >> 4, q = l & 15;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    w.w1[t] = P[OW1 + (16 * t + q) * NIN + g];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      w.b1[t][r] = P[OB1 + 16 * t + 4 * g + r];
      w.b2[t][r] = P[OB2 + 16 * t + 4 * g + r];
      w.w3[t][r] = P[OW3 + 16 * t + 4 * g + r];
    }
  }
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int s = 0; s < 8; ++s) w.w2[m][s] = P[OW2 + (16 * m + q) * H1 + 16 * (s >> 2) + 4 * g + (s & 3)];
  w.b3 = P[OB3];
}

// tanh without branches: 2 / (1 + exp(-2x)) - 1 with the hardware exp2 and
// reciprocal (exp overflowing to +inf for large negative x gives -1); absolute
// error ~2e-7, which is what the weighted sums of the next layer see.
__device__ __forceinline__ float tanh_exp(float x) {
  const float e = __builtin_amdgcn_exp2f(x * -2.8853900817779268f);
  return fmaf(2.0f, __builtin_amdgcn_rcpf(1.0f + e), -1.0f);
}

// Output pre-activation o for a chunk of 64 coefficients, lane l holding the
// four features of coefficient l.  The chunk is four tiles of 16
// coefficients; lane (g, q) takes feature g of coefficient 16t + q of tile t
// (staged through `lds`, this wave's 256 floats) and receives o of
// coefficient l.  The four tiles go through each layer together, so the
// matrix core sees eight independent accumulation chains in the 32x32 layer
// while the VALU works on the tanh of the other tiles.
template <int TB>
__device__ __forceinline__ float net_chunk(const MfmaNet& w, float* lds, const float x[NIN]) {
  const int l = threadIdx.x & 63, g = l >> 4, q = l & 15;
  reinterpret_cast<float4*>(lds)[l] = make_float4(x[0], x[1], x[2], x[3]);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  float xb[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) xb[t] = lds[(16 * t + q) * NIN + g];
  __builtin_amdgcn_wave_barrier();
  float o[4];
#pragma unroll
  for (int t0 = 0; t0 < 4; t0 += TB) {
    f4_t h1[TB][2], h2[TB][2];
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int m = 0; m < 2; ++m)
        h1[t][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(
            w.w1[m], xb[t0 + t], f4_t{w.b1[m][0], w.b1[m][1], w.b1[m][2], w.b1[m][3]}, 0, 0, 0);
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int m = 0; m < 2; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) h1[t][m][r] = tanh_exp(h1[t][m][r]);
        h2[t][m] = f4_t{w.b2[m][0], w.b2[m][1], w.b2[m][2], w.b2[m][3]};
      }
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int m = 0; m < 2; ++m)
          h2[t][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(w.w2[m][s], h1[t][s >> 2][s & 3], h2[t][m], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < TB; ++t) {
      float a = 0.0f;
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) a = fmaf(w.w3[m][r], tanh_exp(h2[t][m][r]), a);
      a += __shfl_xor(a, 16, 64);
      a += __shfl_xor(a, 32, 64);
      o[t0 + t] = a;
    }
  }
  const float mine = g == 0 ? o[0] : g == 1 ? o[1] : g == 2 ? o[2] : o[3];
  return mine + w.b3;
}

// tiles that go through a layer together (register use against overlap)
constexpr int kNetTiles = 2;

constexpr int kNetWaves = 4;   // waves per inference workgroup

__global__ void __launch_bounds__(64 * kNetWaves)
k_forward(const float* __restrict__ P, const float* __restrict__ feat, float* __restrict__ c, long long n) {
  __shared__ float lds[kNetWaves][64 * NIN];
  MfmaNet w;
  load_net(P, w);
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long nch = (n + 63) / 64;
  for (long long ch = blockIdx.x * (long long)kNetWaves + wv; ch < nch; ch += (long long)gridDim.x * kNetWaves) {
    const long long i = ch * 64 + l;
    float x[NIN] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (i < n) {
      const float4 f = reinterpret_cast<const float4*>(feat)[i];
      x[0] = f.x; x[1] = f.y; x[2] = f.z; x[3] = f.w;
    }
    const float o = net_chunk<kNetTiles>(w, lds[wv], x);
    if (i < n) c[i] = softplusf(o) + 1e-6f;
  }
}

// Per-block gradient partials over RB records.  mode 0: dc given (backward of
// sum dc*c); mode 1: records, dc from the loss derivative, loss accumulated.
// scratch[block][0..1248] gradient partials, scratch[block][1249] loss.
template <int MODE>
__global__ void __launch_bounds__(RB)
k_grad_block(const float* __restrict__ params, const float* __restrict__ feat, const float* __restrict__ aux,
             int n, double* __restrict__ scratch) {
  __shared__ float P[MLP_NP];
  __shared__ float xs[NIN][RP], h1s[H1][RP], h2s[H2][RP], d1s[H1][RP], d2s[H2][RP], dos[RP];
  load_params(params, P);
  const int r = threadIdx.x;
  const int idx = blockIdx.x * RB + r;
  float x[NIN] = {0, 0, 0, 0}, h1[H1], h2[H2];
  float dout = 0.0f;
  double e = 0.0;
  if (idx < n) {
    const float4 f = reinterpret_cast<const float4*>(feat)[idx];
    x[0] = f.x; x[1] = f.y; x[2] = f.z; x[3] = f.w;
    const float o = fwd1(P, x, h1, h2);
    float dc;
    if constexpr (MODE == 0) {
      dc = aux[idx];
    } else {
      const float c = softplusf(o) + 1e-6f;
      const float* rc = aux + (long long)idx * MLP_REC;
      const double u = rc[0], p = rc[1], L1 = rc[2], L2 = rc[3], S12 = rc[4], w = rc[5];
      const double D = L1 + S12;
      const double res = u - (double)c * p;
      const double a = (L1 * L1 + L2 * L2) / (D * D);
      e = w * a * res * res;
      dc = (float)(-2.0 * w * a * p * res);
    }
    dout = dc * sigmoidf(o);
  } else {
#pragma unroll
    for (int i = 0; i < H1; ++i) h1[i] = 0.0f;
#pragma unroll
    for (int i = 0; i < H2; ++i) h2[i] = 0.0f;
  }
  // back-propagate to the hidden pre-activations
  float d2[H2];
#pragma unroll
  for (int i = 0; i < H2; ++i) d2[i] = dout * P[OW3 + i] * (1.0f - h2[i] * h2[i]);
#pragma unroll 4
  for (int j = 0; j < H1; ++j) {
    float a = 0.0f;
#pragma unroll
    for (int i = 0; i < H2; ++i) a = fmaf(d2[i], P[OW2 + i * H1 + j], a);
    d1s[j][r] = a * (1.0f - h1[j] * h1[j]);
  }
#pragma unroll
  for (int j = 0; j < NIN; ++j) xs[j][r] = x[j];
#pragma unroll
  for (int i = 0; i < H1; ++i) h1s[i][r] = h1[i];
#pragma unroll
  for (int i = 0; i < H2; ++i) {
    h2s[i][r] = h2[i];
    d2s[i][r] = d2[i];
  }
  dos[r] = dout;
  __syncthreads();
  double* out = scratch + (long long)blockIdx.x * (MLP_NP + 1);
  for (int p = r; p < MLP_NP; p += RB) {
    double g = 0.0;
    if (p < OB1) {
      const int i = p / NIN, j = p % NIN;
      for (int k = 0; k < RB; ++k) g += (double)d1s[i][k] * (double)xs[j][k];
    } else if (p < OW2) {
      const int i = p - OB1;
      for (int k = 0; k < RB; ++k) g += (double)d1s[i][k];
    } else if (p < OB2) {
      const int i = (p - OW2) / H1, j = (p - OW2) % H1;
      for (int k = 0; k < RB; ++k) g += (double)d2s[i][k] * (double)h1s[j][k];
    } else if (p < OW3) {
      const int i = p - OB2;
      for (int k = 0; k < RB; ++k) g += (double)d2s[i][k];
    } else if (p < OB3) {
      const int i = p - OW3;
      for (int k = 0; k < RB; ++k) g += (double)dos[k] * (double)h2s[i][k];
    } else {
      for (int k = 0; k < RB; ++k) g += (double)dos[k];
    }
    out[p] = g;
  }
  e = wave_sum(e);
  if (r == 0) out[MLP_NP] = e;
}

// Sums the block partials in block order.  accumulate: grad += (else =).
__global__ void __launch_bounds__(256)
k_grad_reduce(const double* __restrict__ scratch, int nblk, float* __restrict__ grad, double* __restrict__ loss,
              int accumulate) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p <= MLP_NP; p += gridDim.x * blockDim.x) {
    double g = 0.0;
    for (int b = 0; b < nblk; ++b) g += scratch[(long long)b * (MLP_NP + 1) + p];
    if (p < MLP_NP) {
      grad[p] = accumulate ? (float)((double)grad[p] + g) : (float)g;
    } else if (loss) {
      *loss = g;
    }
  }
}

__global__ void __launch_bounds__(256)
k_adam(float* __restrict__ params, const float* __restrict__ grad, float* __restrict__ m, float* __restrict__ v,
       float b1t, float b2t, float lr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_NP) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.0f - b1t);
  const float vh = vi / (1.0f - b2t);
  params[i] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void __launch_bounds__(256)
k_log_l1(const double* __restrict__ s1, const double* __restrict__ s2, long long n, double* partial) {
  double a = 0.0;
  for (long long i = gtid(); i < n; i += gstride()) a += log(s1[i] + s2[i]);
  __shared__ double red[4];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256)
k_fin_mean(const double* partial, int nb, double scale, double* out) {
  double a = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) a += partial[i];
  __shared__ double red[4];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) *out = (red[0] + red[1] + red[2] + red[3]) * scale;
}

__global__ void __launch_bounds__(256)
k_features(const double* __restrict__ s1, const double* __restrict__ s2, const double* __restrict__ beta,
           const double* __restrict__ diagH, const double* __restrict__ meanlog, const double* __restrict__ bmax,
           float* __restrict__ feat, long long n) {
  const double ml = *meanlog;
  const double bm = *bmax > 0.0 ? *bmax : 1.0;
  for (long long i = gtid(); i < n; i += gstride()) {
    const double L1 = s1[i] + s2[i], L2 = s1[i] - s2[i];
    float4 f;
    f.x = (float)(log(L1) - ml);
    f.y = (float)(L2 / L1);
    f.z = (float)log(fabs(beta[i]) / bm + 1e-12);
    f.w = (float)diagH[i];
    reinterpret_cast<float4*>(feat)[i] = f;
  }
}


// The same two steps computed from the interior-point state, with
// Sigma_j = nu_j / s_j, s1 = z + beta, s2 = z - beta formed on the fly.
__global__ void __launch_bounds__(256)
k_log_l1_state(const double* __restrict__ beta, const double* __restrict__ z, const double* __restrict__ nu1,
               const double* __restrict__ nu2, long long n, double* partial) {
  double a = 0.0;
  for (long long i = gtid(); i < n; i += gstride())
    a += log(nu1[i] / (z[i] + beta[i]) + nu2[i] / (z[i] - beta[i]));
  __shared__ double red[4];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256)
k_features_state(const double* __restrict__ beta, const double* __restrict__ z, const double* __restrict__ nu1,
                 const double* __restrict__ nu2, const double* __restrict__ diagH,
                 const double* __restrict__ meanlog, const double* __restrict__ bmax, float* __restrict__ feat,
                 long long n) {
  const double ml = *meanlog;
  const double bm = *bmax > 0.0 ? *bmax : 1.0;
  for (long long i = gtid(); i < n; i += gstride()) {
    const double b = beta[i];
    const double g1 = nu1[i] / (z[i] + b), g2 = nu2[i] / (z[i] - b);
    const double L1 = g1 + g2, L2 = g1 - g2;
    float4 f;
    f.x = (float)(log(L1) - ml);
    f.y = (float)(L2 / L1);
    f.z = (float)log(fabs(b) / bm + 1e-12);
    f.w = (float)diagH[i];
    reinterpret_cast<float4*>(feat)[i] = f;
  }
}


// Gate and features of coefficient i of the interior-point state.  The
// slacks are formed in FP64 (z and |beta| nearly cancel late in the solve);
// the gate is pc_gate (no division).  The features are FP32 from the FP64
// slacks.  diagH is read only where the gate passes: the network maps each
// coefficient's features to its own output (a column of every layer's
// product), so an inactive lane's features, whose output is discarded, need
// not be exact.
__device__ __forceinline__ bool state_features(const double* __restrict__ beta, const double* __restrict__ z,
                                               const double* __restrict__ nu1, const double* __restrict__ nu2,
                                               const double* __restrict__ diagH, double ml, double ibm,
                                               long long i, float x[NIN]) {
  const double b = beta[i], a1 = nu1[i], a2 = nu2[i];
  const double s1 = z[i] + b, s2 = z[i] - b;
  const bool act = pc_gate(a1, a2, s1, s2);
  const float g1 = (float)a1 * __builtin_amdgcn_rcpf((float)s1);
  const float g2 = (float)a2 * __builtin_amdgcn_rcpf((float)s2);
  const float L1 = g1 + g2;
  x[0] = __logf(L1) - (float)ml;
  x[1] = (g1 - g2) * __builtin_amdgcn_rcpf(L1);
  x[2] = __logf((float)(fabs(b) * ibm) + 1e-12f);
  x[3] = act ? (float)diagH[i] : 0.0f;
  return act;
}

// Correction of the interior-point state in one pass: Sigma_j = nu_j / s_j,
// the four features, and c = softplus(MLP) + 1e-6 only where c can act on
// P_c^{-1}, i.e. where L1 / (L1 + 4 S1 S2) >= kPcRelevance; elsewhere c = 1
// (the paper's P, from which P_c^{-1} then differs by less than that
// relative).  The network runs on the matrix cores for every 64-coefficient
// chunk that holds an active coefficient; set[chunk] records which chunks
// those are (where c may differ from 1).
__global__ void __launch_bounds__(64 * kNetWaves)
k_correction_state(const double* __restrict__ beta, const double* __restrict__ z, const double* __restrict__ nu1,
                   const double* __restrict__ nu2, const double* __restrict__ diagH,
                   const double* __restrict__ meanlog, double mscale, const double* __restrict__ bmax,
                   const float* __restrict__ P, float* __restrict__ c, long long n, uint32_t* __restrict__ set) {
  __shared__ float lds[kNetWaves][64 * NIN];
  MfmaNet w;
  load_net(P, w);
  const double ml = *meanlog * mscale;
  const double ibm = *bmax > 0.0 ? 1.0 / *bmax : 1.0;
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long nch = (n + 63) / 64;
  for (long long ch = blockIdx.x * (long long)kNetWaves + wv; ch < nch; ch += (long long)gridDim.x * kNetWaves) {
    const long long i = ch * 64 + l;
    float x[NIN] = {0.0f, 0.0f, 0.0f, 0.0f};
    const bool act = i < n && state_features(beta, z, nu1, nu2, diagH, ml, ibm, i, x);
    float o = 0.0f;
    const bool any = __ballot(act) != 0;
    if (any) o = net_chunk<kNetTiles>(w, lds[wv], x);   // chunks without an active coefficient skip the network
    if (i < n) c[i] = act ? softplusf(o) + 1e-6f : 1.0f;
    if (l == 0) set[ch] = any ? 1u : 0u;
  }
}

// One active chunk of k_correction_patch: c of its 64 coefficients, the
// patched PCG start where c acts, and the changes of the start sums.
template <typename TC>
__device__ __forceinline__ void patch_chunk(const MfmaNet& w, float* lds, const double* __restrict__ beta,
                                            const double* __restrict__ z, const double* __restrict__ nu1,
                                            const double* __restrict__ nu2, const double* __restrict__ diagH,
                                            double ml, double ibm, float* __restrict__ c, uint32_t* __restrict__ set,
                                            long long n, long long ch, int l, bool h64, const TC* __restrict__ s1c,
                                            const TC* __restrict__ s2c, const TC* __restrict__ rb,
                                            const TC* __restrict__ rz, TC* __restrict__ pb, TC* __restrict__ pz,
                                            const double* __restrict__ s164, const double* __restrict__ s264,
                                            const double* __restrict__ hb64, const double* __restrict__ hz64,
                                            double& d0, double& d1) {
  constexpr bool F64 = std::is_same<TC, double>::value;
  const long long i = ch * kPcChunk + l;
  float x[NIN] = {0.0f, 0.0f, 0.0f, 0.0f};
  const bool a = i < n && state_features(beta, z, nu1, nu2, diagH, ml, ibm, i, x);
  const float o = net_chunk<kNetTiles>(w, lds, x);
  const float ci = a ? softplusf(o) + 1e-6f : 1.0f;
  if (i < n) c[i] = ci;
  if (l == 0) set[ch] = 1u;
  if (a) {
    const double cv = (double)ci;
    const TC r1 = rb[i], r2 = rz[i], g1 = s1c[i], g2 = s2c[i];
    TC w1, w2, v1, v2;
    pinv_block<TC>(r1, r2, g1, g2, cv, w1, w2);
    pinv_block<TC>(r1, r2, g1, g2, 1.0, v1, v2);
    pb[i] = w1;
    pz[i] = w2;
    d0 += ((double)r1 * (double)w1 + (double)r2 * (double)w2) - ((double)r1 * (double)v1 + (double)r2 * (double)v2);
    if constexpr (F64) {
      d1 += (r1 * w1 + r2 * w2) - (r1 * v1 + r2 * v2);
    } else if (h64) {
      const double h1 = hb64[i], h2 = hz64[i], G1 = s164[i], G2 = s264[i];
      double u1, u2, q1, q2;
      pinv_block<double>(h1, h2, G1, G2, cv, u1, u2);
      pinv_block<double>(h1, h2, G1, G2, 1.0, q1, q2);
      d1 += (h1 * u1 + h2 * u2) - (h1 * q1 + h2 * q2);
    }
  }
}

// The correction of an iterate whose Newton system the iterate update has
// already built with the paper's P (c = 1): c as k_correction_state forms
// it, and, at each coefficient where c acts, the PCG start patched in place
// to p = P_c^{-1} r, by the same arithmetic as the Newton build with c.
// Only chunks are visited that the update flagged active (act) or where c
// was last set (set; every chunk when c is not known to be 1 outside them,
// !tracked); set is brought up to date.  Each workgroup adds what the patch
// changes in r.P^{-1}r (quantity 0, in the Krylov precision TC, summed in
// FP64) and in h.P^{-1}h (quantity 1, FP64; only when h64 is given) to its
// own partial of the update's reduction, so the start sums become those of
// the corrected system.  The grid must not exceed the update's workgroup
// count.  For TC = double, r is h and the FP64 Sigma is s1c/s2c; for TC =
// float the FP64 h and Sigma are hb64/hz64 and s164/s264 (null for a system
// solved without refinement, whose h.P^{-1}h is not used).
template <typename TC>
__global__ void __launch_bounds__(64 * kNetWaves)
k_correction_patch(const double* __restrict__ beta, const double* __restrict__ z, const double* __restrict__ nu1,
                   const double* __restrict__ nu2, const double* __restrict__ diagH,
                   const double* __restrict__ meanlog, double mscale, const double* __restrict__ bmax,
                   const float* __restrict__ P, float* __restrict__ c, long long n,
                   const uint32_t* __restrict__ act, uint32_t* __restrict__ set, int tracked,
                   const TC* __restrict__ s1c, const TC* __restrict__ s2c, const TC* __restrict__ rb,
                   const TC* __restrict__ rz, TC* __restrict__ pb, TC* __restrict__ pz,
                   const double* __restrict__ s164, const double* __restrict__ s264,
                   const double* __restrict__ hb64, const double* __restrict__ hz64, double* partial, int stride) {
  constexpr bool F64 = std::is_same<TC, double>::value;
  __shared__ float lds[kNetWaves][64 * NIN];
  __shared__ double red[2][kNetWaves];
  MfmaNet w;
  bool loaded = false;
  const double ml = *meanlog * mscale;
  const double ibm = *bmax > 0.0 ? 1.0 / *bmax : 1.0;
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long nch = (n + kPcChunk - 1) / kPcChunk;
  const bool h64 = F64 || hb64 != nullptr;
  double d0 = 0.0, d1 = 0.0;
  // wave v takes the chunks v, v + W, v + 2W, ... (W waves in the grid);
  // lane l reads the flags of the wave's chunk 64 g + l of that sequence, so
  // one load serves 64 of its chunks, and the wave visits those that need
  // work (the ballot and the visit order are uniform across the wave)
  const long long nwaves = (long long)gridDim.x * kNetWaves;
  const long long first = blockIdx.x * (long long)kNetWaves + wv;
  for (long long g0 = 0; first + g0 * nwaves < nch; g0 += 64) {
    const long long mine = first + (g0 + l) * nwaves;
    bool isact = false, need = false;
    if (mine < nch) {
      isact = act[mine] != 0u;
      need = isact || !tracked || set[mine] != 0u;
    }
    unsigned long long todo = __ballot(need);
    const unsigned long long acts = __ballot(isact);
    while (todo) {
      const int b = __ffsll((long long)todo) - 1;
      todo &= todo - 1ull;
      const long long ch = first + (g0 + b) * nwaves;
      const long long i = ch * kPcChunk + l;
      if (!((acts >> b) & 1ull)) {
        if (i < n) c[i] = 1.0f;
        if (l == 0) set[ch] = 0u;
        continue;
      }
      if (!loaded) {
        load_net(P, w);
        loaded = true;
      }
      patch_chunk<TC>(w, lds[wv], beta, z, nu1, nu2, diagH, ml, ibm, c, set, n, ch, l, h64, s1c, s2c, rb, rz, pb,
                      pz, s164, s264, hb64, hz64, d0, d1);
    }
  }
  d0 = wave_sum(d0);
  d1 = wave_sum(d1);
  if (l == 0) {
    red[0][wv] = d0;
    red[1][wv] = d1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = 0.0, a1 = 0.0;
    for (int k = 0; k < kNetWaves; ++k) {
      a0 += red[0][k];
      a1 += red[1][k];
    }
    partial[blockIdx.x] += a0;
    if (h64) partial[stride + blockIdx.x] += a1;
  }
}

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Records at coefficients i_j, j < npick: i_j = splitmix64(seed + j) mod n,
// or, with a list of the m = *count coefficients where the correction can
// act (idx), i_j = idx[splitmix64(seed + j) mod m]; with an empty list every
// record has p = 0 and carries no weight.
template <typename T>
__global__ void __launch_bounds__(256)
k_capture(const T* __restrict__ pb, const T* __restrict__ pz, const T* __restrict__ qb, const T* __restrict__ qz,
          const T* __restrict__ s1, const T* __restrict__ s2, const float* __restrict__ feat_all, long long n,
          int npick, unsigned long long seed, const int* __restrict__ idx, const long long* __restrict__ count,
          float* __restrict__ of, float* __restrict__ orc, double* partial) {
  (void)qz;   // (H p) is the beta row of q less its Sigma terms; q_z is not needed
  const long long m = idx ? *count : n;
  double acc = 0.0;
  for (long long j = gtid(); j < npick; j += gstride()) {
    float* rc = orc + j * MLP_REC;
    if (m == 0) {
      rc[0] = 0.0f; rc[1] = 0.0f; rc[2] = 1.0f; rc[3] = 0.0f; rc[4] = 0.0f; rc[5] = 1.0f;
      reinterpret_cast<float4*>(of)[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      continue;
    }
    const long long h = (long long)(splitmix64(seed + (unsigned long long)j) % (unsigned long long)m);
    const long long i = idx ? (long long)idx[h] : h;
    const double b = pb[i], z = pz[i], g1 = s1[i], g2 = s2[i];
    const double u = (double)qb[i] - g1 * (b + z) - g2 * (b - z);
    rc[0] = (float)u;
    rc[1] = (float)b;
    rc[2] = (float)(g1 + g2);
    rc[3] = (float)(g1 - g2);
    rc[4] = (float)(4.0 * g1 * g2);
    rc[5] = 1.0f;
    reinterpret_cast<float4*>(of)[j] = reinterpret_cast<const float4*>(feat_all)[i];
    acc += b * b + z * z;
  }
  __shared__ double red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// The coefficients where the correction can act, L1 / (L1 + 4 S1 S2) >= rmin
// from the barrier diagonals, listed in increasing order: each of nb
// workgroups counts its contiguous range, one workgroup turns the counts into
// offsets, and each range is written out in order (wave ballots for the
// order within a round of 256).
template <typename T>
__device__ __forceinline__ bool sigma_gate(const T* s1, const T* s2, long long i, double rmin) {
  const double g1 = s1[i], g2 = s2[i], L1 = g1 + g2;
  return L1 >= rmin * (L1 + 4.0 * g1 * g2);
}

__device__ __forceinline__ void gate_range(long long n, long long& lo, long long& hi) {
  const long long per = (n + gridDim.x - 1) / gridDim.x;
  lo = blockIdx.x * per;
  hi = lo + per < n ? lo + per : n;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_gate_count(const T* __restrict__ s1, const T* __restrict__ s2, long long n, double rmin, int* __restrict__ counts) {
  long long lo, hi;
  gate_range(n, lo, hi);
  int k = 0;
  for (long long i = lo + threadIdx.x; i < hi; i += 256) k += sigma_gate(s1, s2, i, rmin) ? 1 : 0;
  __shared__ int red[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) k += __shfl_xor(k, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = k;
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(64)
k_gate_scan(int* __restrict__ counts, int nb, long long* __restrict__ total) {
  if (threadIdx.x != 0) return;
  long long acc = 0;
  for (int b = 0; b < nb; ++b) {
    const int k = counts[b];
    counts[b] = (int)acc;
    acc += k;
  }
  *total = acc;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_gate_compact(const T* __restrict__ s1, const T* __restrict__ s2, long long n, double rmin,
               const int* __restrict__ offsets, int* __restrict__ idx) {
  long long lo, hi;
  gate_range(n, lo, hi);
  __shared__ int wsum[4];
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  long long base = offsets[blockIdx.x];
  for (long long r = lo; r < hi; r += 256) {
    const long long i = r + threadIdx.x;
    const bool act = i < hi && sigma_gate(s1, s2, i, rmin);
    const unsigned long long m = __ballot(act);
    if (l == 0) wsum[wv] = __popcll(m);
    __syncthreads();
    int before = 0;
    for (int k = 0; k < wv; ++k) before += wsum[k];
    const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (act) idx[base + before + __popcll(m & ((1ull << l) - 1ull))] = (int)i;
    base += total;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256)
k_set_weights(float* __restrict__ rec, int npick, const double* __restrict__ total) {
  const double t = *total;
  const float w = t > 0.0 ? (float)(1.0 / t) : 0.0f;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < npick; j += gridDim.x * blockDim.x) rec[j * MLP_REC + 5] = w;
}

__global__ void __launch_bounds__(256)
k_scale_weights(float* __restrict__ rec, int npick, float f) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < npick; j += gridDim.x * blockDim.x) rec[j * MLP_REC + 5] *= f;
}

// inference grid: one 64-coefficient chunk per wave and round, at most
// 2560 workgroups (10 per compute unit)
int net_blocks(long long n) {
  long long b = ((n + 63) / 64 + kNetWaves - 1) / kNetWaves;
  if (b > 2560) b = 2560;
  if (b < 1) b = 1;
  return (int)b;
}

int blocks_for(long long n) {
  long long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

void mlp_mean_log_l1(const double* s1, const double* s2, long long n, double* partial, double* out, hipStream_t s) {
  const int nb = blocks_for(n);
  hipLaunchKernelGGL(k_log_l1, dim3(nb), dim3(256), 0, s, s1, s2, n, partial);
  hipLaunchKernelGGL(k_fin_mean, dim3(1), dim3(256), 0, s, partial, nb, 1.0 / (double)n, out);
}

void mlp_features(const double* s1, const double* s2, const double* beta, const double* diagH, const double* meanlog,
                  const double* bmax, float* feat, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3(blocks_for(n)), dim3(256), 0, s, s1, s2, beta, diagH, meanlog, bmax, feat, n);
}

void mlp_features_state(const double* beta, const double* z, const double* nu1, const double* nu2,
                        const double* diagH, const double* bmax, float* feat, long long n, double* partial,
                        double* meanlog, hipStream_t s) {
  const int nb = blocks_for(n);
  hipLaunchKernelGGL(k_log_l1_state, dim3(nb), dim3(256), 0, s, beta, z, nu1, nu2, n, partial);
  hipLaunchKernelGGL(k_fin_mean, dim3(1), dim3(256), 0, s, partial, nb, 1.0 / (double)n, meanlog);
  hipLaunchKernelGGL(k_features_state, dim3(nb), dim3(256), 0, s, beta, z, nu1, nu2, diagH, (const double*)meanlog,
                     bmax, feat, n);
}

void mlp_mean_log_l1_state(const double* beta, const double* z, const double* nu1, const double* nu2, long long n,
                           double* partial, double* meanlog, hipStream_t s) {
  const int nb = blocks_for(n);
  hipLaunchKernelGGL(k_log_l1_state, dim3(nb), dim3(256), 0, s, beta, z, nu1, nu2, n, partial);
  hipLaunchKernelGGL(k_fin_mean, dim3(1), dim3(256), 0, s, partial, nb, 1.0 / (double)n, meanlog);
}

void mlp_correction_state(const double* beta, const double* z, const double* nu1, const double* nu2,
                          const double* diagH, const double* meanlog, double mscale, const double* bmax,
                          const float* params, float* c, long long n, uint32_t* set, hipStream_t s) {
  hipLaunchKernelGGL(k_correction_state, dim3(net_blocks(n)), dim3(64 * kNetWaves), 0, s, beta, z, nu1, nu2, diagH,
                     meanlog, mscale, bmax, params, c, n, set);
}

template <typename TC>
void mlp_correction_patch(const double* beta, const double* z, const double* nu1, const double* nu2,
                          const double* diagH, const double* meanlog, double mscale, const double* bmax,
                          const float* params, float* c, long long n, const uint32_t* act, uint32_t* set,
                          bool tracked, const TC* s1c, const TC* s2c, const TC* rb, const TC* rz, TC* pb, TC* pz,
                          const double* s164, const double* s264, const double* hb64, const double* hz64,
                          double* partial, int stride, int max_blocks, hipStream_t s) {
  const int nb = std::max(1, std::min(net_blocks(n), max_blocks));
  hipLaunchKernelGGL(k_correction_patch<TC>, dim3(nb), dim3(64 * kNetWaves), 0, s, beta, z, nu1, nu2, diagH, meanlog,
                     mscale, bmax, params, c, n, act, set, tracked ? 1 : 0, s1c, s2c, rb, rz, pb, pz, s164, s264,
                     hb64, hz64, partial, stride);
}
template void mlp_correction_patch<float>(const double*, const double*, const double*, const double*, const double*,
                                          const double*, double, const double*, const float*, float*, long long,
                                          const uint32_t*, uint32_t*, bool, const float*, const float*, const float*,
                                          const float*, float*, float*, const double*, const double*, const double*,
                                          const double*, double*, int, int, hipStream_t);
template void mlp_correction_patch<double>(const double*, const double*, const double*, const double*, const double*,
                                           const double*, double, const double*, const float*, float*, long long,
                                           const uint32_t*, uint32_t*, bool, const double*, const double*,
                                           const double*, const double*, double*, double*, const double*,
                                           const double*, const double*, const double*, double*, int, int,
                                           hipStream_t);

void mlp_forward(const float* params, const float* feat, float* c, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_forward, dim3(net_blocks(n)), dim3(64 * kNetWaves), 0, s, params, feat, c, n);
}

void mlp_backward(const float* params, const float* feat, const float* dc, float* grad, int n, double* scratch,
                  hipStream_t s) {
  const int nblk = (n + RB - 1) / RB;
  hipLaunchKernelGGL((k_grad_block<0>), dim3(nblk), dim3(RB), 0, s, params, feat, dc, n, scratch);
  hipLaunchKernelGGL(k_grad_reduce, dim3((MLP_NP + 256) / 256), dim3(256), 0, s, scratch, nblk, grad,
                     (double*)nullptr, 1);
}

void mlp_loss_grad(const float* params, const float* feat, const float* rec, int n, double* loss, float* grad,
                   double* scratch, hipStream_t s) {
  const int nblk = (n + RB - 1) / RB;
  hipLaunchKernelGGL((k_grad_block<1>), dim3(nblk), dim3(RB), 0, s, params, feat, rec, n, scratch);
  hipLaunchKernelGGL(k_grad_reduce, dim3((MLP_NP + 256) / 256), dim3(256), 0, s, scratch, nblk, grad, loss, 0);
}

void mlp_adam(float* params, const float* grad, float* m, float* v, int t, float lr, hipStream_t s) {
  const float b1t = (float)std::pow(0.9, (double)t);
  const float b2t = (float)std::pow(0.999, (double)t);
  hipLaunchKernelGGL(k_adam, dim3((MLP_NP + 255) / 256), dim3(256), 0, s, params, grad, m, v, b1t, b2t, lr);
}

template <typename T>
void mlp_capture(const T* pb, const T* pz, const T* qb, const T* qz, const T* s1, const T* s2, const float* feat_all,
                 long long n, int npick, unsigned long long seed, float* out_feat, float* out_rec, double* partial,
                 int* gate_idx, double rmin, hipStream_t s) {
  const int* idx = nullptr;
  long long* count = nullptr;
  if (gate_idx) {
    // the counts and their total sit past the capture's own partials
    int* counts = reinterpret_cast<int*>(partial + 8192);
    count = reinterpret_cast<long long*>(partial + 8192 + kGateBlocks / 2);
    const int gb = (int)std::max(1LL, std::min<long long>(kGateBlocks, (n + 255) / 256));
    hipLaunchKernelGGL((k_gate_count<T>), dim3(gb), dim3(256), 0, s, s1, s2, n, rmin, counts);
    hipLaunchKernelGGL(k_gate_scan, dim3(1), dim3(64), 0, s, counts, gb, count);
    hipLaunchKernelGGL((k_gate_compact<T>), dim3(gb), dim3(256), 0, s, s1, s2, n, rmin, (const int*)counts, gate_idx);
    idx = gate_idx;
  }
  const int nb = blocks_for(npick);
  hipLaunchKernelGGL((k_capture<T>), dim3(nb), dim3(256), 0, s, pb, pz, qb, qz, s1, s2, feat_all, n, npick, seed,
                     idx, (const long long*)count, out_feat, out_rec, partial);
  double* total = partial + 4096;
  hipLaunchKernelGGL(k_fin_mean, dim3(1), dim3(256), 0, s, partial, nb, 1.0, total);
  hipLaunchKernelGGL(k_set_weights, dim3(blocks_for(npick)), dim3(256), 0, s, out_rec, npick, (const double*)total);
}

void mlp_scale_weights(float* rec, int npick, float factor, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_weights, dim3(blocks_for(npick)), dim3(256), 0, s, rec, npick, factor);
}

template void mlp_capture<double>(const double*, const double*, const double*, const double*, const double*,
                                  const double*, const float*, long long, int, unsigned long long, float*, float*,
                                  double*, int*, double, hipStream_t);
template void mlp_capture<float>(const float*, const float*, const float*, const float*, const float*, const float*,
                                 const float*, long long, int, unsigned long long, float*, float*, double*, int*,
                                 double, hipStream_t);

}  // namespace csipm
