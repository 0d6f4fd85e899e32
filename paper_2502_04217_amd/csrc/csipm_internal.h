// Internal declarations of the csipm HIP library (gfx950).
//
// Data layout on the device ("internal layout").  Every beta-indexed vector
// (beta, z, nu1, nu2, xi, the barrier diagonals, Krylov vectors) is stored as
// n reals that reinterpret as a complex array P[k1][k2][m], m in [0, N3/2):
//   m >= 1 : P = (beta[k1,k2,m], beta[-k1,-k2,N3-m])   (sqrt2 Re / sqrt2 Im of
//            the half-spectrum bin (k1,k2,m))
//   m == 0 : P = (beta[k1,k2,0], beta[k1,k2,N3/2])      (the two self-paired
//            planes k3 = 0 and k3 = N3/2, packed as real/imaginary parts)
// This is a pure permutation of the external row-major beta layout, so all
// elementwise interior-point arithmetic and every dot product are unchanged;
// only the FFT passes see the complex structure.  The same n reals also hold
// the FFT intermediates: after the two inverse complex passes the array is
// T[j1][j2][m] (packed half-spectrum along axis 3, DC and Nyquist sharing
// slot 0), and after the axis-3 pass it reinterprets as the real grid
// x[j1][j2][j3].
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>

namespace csipm {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

// sum, max and min over the 64 lanes of a wave (every lane gets the result)
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
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.re, -a.im}; }
// multiply by +i (dir > 0) or -i (dir < 0)
template <int DIR, typename T>
__device__ __forceinline__ cx<T> cmul_i(cx<T> a) {
  if constexpr (DIR > 0) return {-a.im, a.re};
  else return {a.im, -a.re};
}

// exp(DIR * 2 pi i k / 16) for k in [0, 16), as literals (k = 0..15).
template <typename T>
__device__ __forceinline__ cx<T> w16(int k, int dir) {
  constexpr double C1 = 0.92387953251128675613;  // cos(pi/8)
  constexpr double S1 = 0.38268343236508977173;  // sin(pi/8)
  constexpr double H = 0.70710678118654752440;   // cos(pi/4)
  const double c[16] = {1, C1, H, S1, 0, -S1, -H, -C1, -1, -C1, -H, -S1, 0, S1, H, C1};
  const double s[16] = {0, S1, H, C1, 1, C1, H, S1, 0, -S1, -H, -C1, -1, -C1, -H, -S1};
  return {T(c[k & 15]), T(dir > 0 ? s[k & 15] : -s[k & 15])};
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }
constexpr int bitrev(int x, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1) << (bits - 1 - i);
  return r;
}

// In-register DFT of size R (power of two, R <= 16; odd sizes 3, 5 and 7
// are dft_odd in fft_kernels.h) in natural order:
// out[k] = sum_j v[j] exp(DIR 2 pi i j k / R).  Iterative radix-2 with the
// bit-reversal done at compile time; trivial twiddles are special-cased.
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_reg(cx<T>* v) {
  constexpr int B = ilog2(R);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int j = bitrev(i, B);
    if (j > i) {
      cx<T> t = v[i];
      v[i] = v[j];
      v[j] = t;
    }
  }
#pragma unroll
  for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
    for (int i = 0; i < R; i += len) {
#pragma unroll
      for (int k = 0; k < len / 2; ++k) {
        cx<T> a = v[i + k];
        cx<T> b = v[i + k + len / 2];
        if (k == 0) {
        } else if (4 * k == len) {
          b = cmul_i<DIR>(b);
        } else {
          b = cmul(b, w16<T>(k * (16 / len), DIR));
        }
        v[i + k] = cadd(a, b);
        v[i + k + len / 2] = csub(a, b);
      }
    }
  }
}

// ---------------------------------------------------------------- plans ----

// Twiddle tables for one grid, in both precisions: tw_L[q] = exp(-2 pi i q/L)
// for L in {N1, N2, M = N3/2, N3}.
template <typename T>
struct Twiddles {
  const cx<T>* t1;   // length N1
  const cx<T>* t2;   // length N2
  const cx<T>* tm;   // length M
  const cx<T>* t3;   // length N3
};

// An even N3 gives the half-spectrum layout (n = n1*n2*n3 reals = n1*n2*m
// complex).  An odd N3 has no Nyquist plane to pack beside the DC plane, so
// its beta-space vectors keep the external order, the transforms run on the
// full Hermitian spectrum (n1*n2*n3 complex), and when n1*n2*n3 is odd one
// more coordinate with no data (a zero column of A) makes the vector length
// n even for the pairwise kernels; the LASSO sets it to 0.
struct Grid {
  int n1, n2, n3, m;   // m = n3/2 (even N3)
  long long n;         // beta-space length: nr, or nr + 1 when nr is odd
  long long nr;        // real-space samples n1*n2*n3
  bool odd3() const { return (n3 & 1) != 0; }
};
inline Grid make_grid(int n1, int n2, int n3) {
  Grid g{n1, n2, n3, n3 / 2, 0, (long long)n1 * n2 * n3};
  g.n = g.nr + (g.nr & 1);
  return g;
}

// 3D class of a frequency under the parametrisation's choice of
// representatives: 0 self-conjugate, 1 canonical, 2 mirror of one.
__device__ __forceinline__ int cls3(int k1, int k2, int k3, int n1, int n2, int n3) {
  const bool e1 = k1 == 0 || 2 * k1 == n1, e2 = k2 == 0 || 2 * k2 == n2, e3 = k3 == 0 || 2 * k3 == n3;
  if (e1 && e2 && e3) return 0;
  if (k3 >= 1 && 2 * k3 < n3) return 1;
  if (e3 && k2 >= 1 && 2 * k2 < n2) return 1;
  if (e3 && e2 && k1 >= 1 && 2 * k1 < n1) return 1;
  return 2;
}

// Selects what the axis-3 pass does.
enum Axis3Mode { A3_C2R = 1, A3_R2C = 2, A3_FULL = 3 };

// Epilogue of the last forward pass (axis 1).
enum EpiMode {
  EPI_NONE = 0,   // write the transform result (A^T x or H p), m = 0 left raw
  EPI_K = 1,      // q = K p with the barrier diagonals, plus p.q partials
  EPI_R = 2       // FP64 only: H d_beta out and r.P^{-1}r of r = h - K d
};

// the learned correction is evaluated where L1 / (L1 + 4 S1 S2) >= this
// (elsewhere the 2x2 block of P_c does not depend on c to this precision)
constexpr double kPcRelevance = 1e-3;
// coefficients per activity flag of the correction (one wave's chunk)
constexpr int kPcChunk = 64;

// The correction's gate at a coefficient with multipliers a1, a2 and slacks
// s1, s2 > 0: L1 / (L1 + 4 S1 S2) >= kPcRelevance with S_j = a_j / s_j,
// multiplied through by s1 s2.  Every operation is rounded on its own (no
// contraction into fused multiply-adds), so that the kernels that evaluate
// it (the residual count, the update's activity flags, the correction)
// decide alike on the same values.
__device__ __forceinline__ bool pc_gate(double a1, double a2, double s1, double s2) {
  const double num = __dadd_rn(__dmul_rn(a1, s2), __dmul_rn(a2, s1));
  const double den = __dadd_rn(num, __dmul_rn(4.0, __dmul_rn(a1, a2)));
  return num >= __dmul_rn(kPcRelevance, den);
}

// CG direction update p <- z + beta p fused into the K-apply of the new p
// (zb null: none).  The passes that first read p apply it and write p back:
// the axis-1 inverse pass to p_beta, the K epilogue to p_z.  Every element
// is updated exactly once.
template <typename T>
struct PUpd {
  T* pb;
  T* pz;
  const T* zb;
  const T* zz;
  const double* beta;   // device scalar
};

template <typename T>
struct KArgs {
  const T* pb;        // p_beta (internal layout)
  const T* pz;        // p_z
  const T* sig1;      // Sigma_1
  const T* sig2;      // Sigma_2
  T* qb;
  T* qz;
  PUpd<T> u;          // fused direction update (u.zb null: none)
};

struct RArgs {
  const double* db;   // d_beta, d_z: the current correction (K input)
  const double* dz;
  const double* sig1;
  const double* sig2;
  const double* hb;   // right-hand side
  const double* hz;
  const float* c;     // learned correction or null (c = 1)
  double* hd;         // out: H d_beta, the transform output
};

// Epilogue arguments: quantity q of block b goes to partial[q * pstride + b].
template <typename T>
struct EpiArgs {
  KArgs<T> k;
  RArgs r;
  double* partial;
  int pstride;
};

// One element of q = K p in Sigma form:
//   q_b = h + S1 (p_b + p_z) + S2 (p_b - p_z),  q_z = S1 (p_b + p_z) - S2 (p_b - p_z)
template <typename T>
__device__ __forceinline__ void k_block(T h, T pb, T pz, T s1, T s2, T& qb, T& qz) {
  const T a = pb + pz, d = pb - pz;
  qb = h + s1 * a + s2 * d;
  qz = s1 * a - s2 * d;
}

// One 2x2 block of P_c^{-1} (equation "invprecond1" with C = diag(c)):
//   [zb; zz] = [[L1, -L2], [-L2, c + L1]] [rb; rz] / (c L1 + 4 S1 S2),
// coefficients formed in double.
template <typename T>
__device__ __forceinline__ void pinv_block(T rb, T rz, T s1, T s2, double c, T& zb, T& zz) {
  const double S1 = (double)s1, S2 = (double)s2;
  const double L1 = S1 + S2, L2 = S1 - S2;
  const double inv = 1.0 / (c * L1 + 4.0 * S1 * S2);
  zb = (T)((L1 * (double)rb - L2 * (double)rz) * inv);
  zz = (T)((-L2 * (double)rb + (c + L1) * (double)rz) * inv);
}

// One 2x2 block of P_c itself (equation "precond1" with C = diag(c)):
//   [qb; qz] = [[c + L1, L2], [L2, L1]] [zb; zz], in double.
template <typename T>
__device__ __forceinline__ void p_block(T zb, T zz, T s1, T s2, double c, double& qb, double& qz) {
  const double L1 = (double)s1 + (double)s2, L2 = (double)s1 - (double)s2;
  qb = (c + L1) * (double)zb + L2 * (double)zz;
  qz = L2 * (double)zb + L1 * (double)zz;
}

// FFT driver entry points (fft.hip).  All work is queued on `s`.
// `skip` (nullable device int): when nonzero at launch time the kernel
// returns at once; lets a batch of Krylov iterations be queued ahead.
// The axis-1 passes also map the m = 0 plane between the real
// parametrisation and the spectrum (inverse: on input; forward: on output,
// before the epilogue); the axis-1 inverse pass applies the direction update
// ea->k.u when ea is set and ea->k.u.zb is not null.
template <typename T>
void launch_axis12(const Grid& g, int axis, int dir, const T* src, T* dst, const Twiddles<T>& tw,
                   int epi, const EpiArgs<T>* ea, const int* skip, hipStream_t s);
template <typename T>
void launch_axis3(const Grid& g, int mode, const T* src, T* dst, const uint32_t* maskbits,
                  const Twiddles<T>& tw, const int* skip, hipStream_t s);
// workgroups of a strided pass (axis 1 or 2, complex size elem_bytes, dir +1
// inverse / -1 forward), those of the m = 0 plane included; for the axis-1
// forward pass also its partial count
int axis12_blocks(const Grid& g, int axis, int elem_bytes, int dir);
// whether the FFT passes have kernels for extent N on `axis` (1, 2: pencils
// of length N; 3: half length N/2 for an even N, full length for an odd N,
// which takes the full-spectrum transforms): every N = 2^a 3^b 5^c 7^d in
// [3, 1024] (instantiated register-resident kernels for the powers of two
// and the lengths fft_mixed_f64/f32.hip list, the LDS-resident kernels of
// fft_any.hip for the rest), and on axes 1 and 2 also 1 and 2 (2D and 1D
// grids)
bool fft_extent_supported(int N, int axis);

// Full-spectrum transforms of a grid with an odd N3 (Grid::odd3): beta in
// external order, work holds n1*n2*n3 complex values.  Each launch returns at
// once when *skip is set.
constexpr int kCpMaxBlocks = 1024;
// workgroups (and partials) of cp_unmap
int cp_blocks(const Grid& g);
// work = B^H beta (the Hermitian spectrum of the real parametrisation)
template <typename T>
void cp_map(const Grid& g, const T* beta, T* work, const int* skip, hipStream_t s);
// p <- z + beta p (both halves; the CG direction update before a K-apply)
template <typename T>
void cp_pupdate(const Grid& g, T* pb, T* pz, const T* zb, const T* zz, const double* beta, const int* skip,
                hipStream_t s);
// unnormalised complex FFT of work along axes 1, 2, 3 (dir +1: inverse,
// exp(+); dir -1: forward, along 3, 2, 1)
template <typename T>
void cp_passes(const Grid& g, int dir, T* work, const Twiddles<T>& tw, const int* skip, hipStream_t s);
// work = mask * Re(work) / nr (the normalisations of an inverse and a
// forward unitary transform), imaginary part 0
template <typename T>
void cp_mask(const Grid& g, T* work, const uint32_t* bits, const int* skip, hipStream_t s);
// x = Re(work) / sqrt(nr); work = x / sqrt(nr)
template <typename T>
void cp_real(const Grid& g, const T* work, T* x, hipStream_t s);
template <typename T>
void cp_cplx(const Grid& g, const T* x, T* work, hipStream_t s);
// the real parametrisation of the spectrum in work: written to out
// (EPI_NONE) or handed to the K / refinement epilogue of ea (EPI_K, EPI_R;
// ea->k.u is ignored, cp_pupdate applies it); returns the partial count
template <typename T>
int cp_unmap(const Grid& g, const T* work, T* out, int epi, const EpiArgs<T>* ea, const int* skip, hipStream_t s);

// message of the last failed context-free call on this thread (noalloc.hip)
const char* noctx_last_error();
void noctx_set_error(const std::string& msg);

// permutation between the external beta layout and the internal one
template <typename Te, typename Ti>
void launch_to_internal(const Grid& g, const Te* ext, Ti* in, hipStream_t s);
template <typename Ti, typename Te>
void launch_to_external(const Grid& g, const Ti* in, Te* ext, hipStream_t s);
void launch_pack_mask(const Grid& g, const uint8_t* obs, uint32_t* bits, hipStream_t s);
// [n][4] float records, internal coefficient order -> external order
void launch_feat_to_external(const Grid& g, const float* in, float* ext, hipStream_t s);

}  // namespace csipm
