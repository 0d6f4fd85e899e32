// Hand-written 3D real FFT passes for the operators A, A^T, H = A^T D A and
// the condensed KKT operator K (paper: "Matrix-free operators" and equation
// "condensedkkt").  gfx950, wave64.
//
// One apply of H is five volume passes over the n-real internal array:
//   axis 1   : inverse complex FFT along k1 (strided pencils); the lanes of
//              the m = 0 plane, whose real parametrisation pairs (k1, k2)
//              with (-k1, -k2), mix the pairs on input
//   axis 2   : inverse complex FFT along k2 (strided pencils)
//   axis 3   : c2r along k3, mask, r2c along k3 (contiguous pencils), using
//              a half-length complex FFT with the DC/Nyquist pair packed in
//              slot 0
//   axis 2   : forward complex FFT along k2
//   axis 1   : forward complex FFT along k1, unmixing the m = 0 pairs, fused
//              with the K epilogue q = K p and the p.q partial sums
// The pencil FFT kernels (Stockham stages, fft_kernels.h) are instantiated
// here for power-of-two lengths and in fft_mixed_f64/f32.hip for lengths with odd
// factors; fft_any.hip serves the other 7-smooth lengths.  Strided passes map consecutive lanes to consecutive pencils, so
// every global access is a run of TM contiguous complex numbers.
#include "fft_kernels.h"

#include <cmath>
#include <type_traits>

namespace csipm {

namespace fftk {
CSIPM_MIXED_INSTANCES(extern, double)
CSIPM_MIXED_INSTANCES(extern, float)
CSIPM_MIXED_INST12(extern, double, 1, -1, EpiR)
}  // namespace fftk

using namespace fftk;

namespace {

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

// With an odd N3 the internal order is the external one, and the internal
// vector has n >= nr entries: the coordinate nr, when there is one, has no
// external counterpart and enters as 0.
__device__ __forceinline__ long long ext_of(long long r, int n1, int n2, int n3, int m) {
  return (n3 & 1) ? r : ext_index(r, n1, n2, n3, m);
}

template <typename Te, typename Ti>
__global__ void k_to_internal(const Te* __restrict__ ext, Ti* __restrict__ in, long long n, long long nr, int n1,
                              int n2, int n3, int m) {
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < n;
       r += (long long)gridDim.x * blockDim.x)
    in[r] = r < nr ? (Ti)ext[ext_of(r, n1, n2, n3, m)] : (Ti)0;
}

template <typename Ti, typename Te>
__global__ void k_to_external(const Ti* __restrict__ in, Te* __restrict__ ext, long long nr, int n1,
                              int n2, int n3, int m) {
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < nr;
       r += (long long)gridDim.x * blockDim.x)
    ext[ext_of(r, n1, n2, n3, m)] = (Te)in[r];
}

__global__ void k_feat_to_external(const float4* __restrict__ in, float4* __restrict__ ext, long long nr, int n1,
                                   int n2, int n3, int m) {
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < nr;
       r += (long long)gridDim.x * blockDim.x)
    ext[ext_of(r, n1, n2, n3, m)] = in[r];
}

__global__ void k_pack_mask(const uint8_t* __restrict__ obs, uint32_t* __restrict__ bits, long long nwords,
                            long long n) {
  for (long long w = blockIdx.x * (long long)blockDim.x + threadIdx.x; w < nwords;
       w += (long long)gridDim.x * blockDim.x) {
    uint32_t v = 0;
    for (int b = 0; b < 32 && w * 32 + b < n; ++b) v |= (obs[w * 32 + b] ? 1u : 0u) << b;
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
                     int m, int n2, Epi epi, const int* skip, hipStream_t s) {
#define CSIPM_A12(LL)                                                                     \
  case LL:                                                                                \
    launch_axis12_at<T, LL, AX, DIR, Epi>(grid, src, dst, geo, tw, m, n2, epi, skip, s); \
    break;
  switch (L) {
    CSIPM_A12(1)
    CSIPM_A12(2)
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
      if (!launch_axis12_mixed<T, AX, DIR, Epi>(L, grid, src, dst, geo, tw, m, n2, epi, skip, s))
        (void)launch_axis12_any<T, AX, DIR, Epi>(L, grid, src, dst, geo, tw, m, n2, epi, skip, s);
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

// ------------------------------------------------ odd N3: full spectrum --
// With an odd N3 the operators run on the whole spectrum: beta (external
// order) is mapped to the Hermitian spectrum W = B^H beta (derivation
// "map"), the three axes are inverse-transformed as complex pencils, the real
// part is masked, the three axes are forward-transformed, and the real
// parametrisation is read back elementwise, since the spectrum of a real
// grid is Hermitian: y_k = sqrt2 Re Y_k (canonical), -sqrt2 Im Y_k (mirror),
// Re Y_k (self-conjugate).  Twice the bytes of the half-spectrum passes;
// grids with an odd N3 are the small odd-N cases.

// class of the flat frequency f = (k1 N2 + k2) N3 + k3 and the flat index of -k
__device__ __forceinline__ int cp_freq(long long f, int n1, int n2, int n3, long long& mf) {
  const int k3 = (int)(f % n3);
  const long long r = f / n3;
  const int k2 = (int)(r % n2);
  const int k1 = (int)(r / n2);
  const int m1 = k1 ? n1 - k1 : 0, m2 = k2 ? n2 - k2 : 0, m3 = k3 ? n3 - k3 : 0;
  mf = ((long long)m1 * n2 + m2) * n3 + m3;
  return cls3(k1, k2, k3, n1, n2, n3);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_cp_map(const T* __restrict__ beta, cx<T>* __restrict__ w, long long nr, int n1, int n2, int n3,
         const int* skip) {
  if (skip && *skip) return;
  const T rs2 = (T)0.70710678118654752440;
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < nr; f += (long long)gridDim.x * blockDim.x) {
    long long mf;
    const int c = cp_freq(f, n1, n2, n3, mf);
    const T b = beta[f];
    if (c == 0) {
      w[f] = {b, (T)0};
    } else {
      const T bm = beta[mf];
      w[f] = c == 1 ? cx<T>{rs2 * b, rs2 * bm} : cx<T>{rs2 * bm, -rs2 * b};
    }
  }
}

// p <- z + beta p on both halves (the CG direction update, which the
// half-spectrum path applies inside its first and last passes)
template <typename T>
__global__ void __launch_bounds__(256)
k_cp_pupd(T* __restrict__ pb, T* __restrict__ pz, const T* __restrict__ zb, const T* __restrict__ zz,
          const double* __restrict__ beta, long long n, const int* skip) {
  if (skip && *skip) return;
  const T be = (T)*beta;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    pb[i] = zb[i] + be * pb[i];
    pz[i] = zz[i] + be * pz[i];
  }
}

// x = Re(w) on the observed samples, 0 elsewhere, scaled (both unitary
// normalisations of H at once); the imaginary part is round-off
template <typename T>
__global__ void __launch_bounds__(256)
k_cp_mask(cx<T>* __restrict__ w, const uint32_t* __restrict__ bits, long long nr, T scale, const int* skip) {
  if (skip && *skip) return;
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < nr; f += (long long)gridDim.x * blockDim.x) {
    const bool o = (bits[f >> 5] >> (f & 31)) & 1u;
    w[f] = {o ? w[f].re * scale : (T)0, (T)0};
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_cp_real(const cx<T>* __restrict__ w, T* __restrict__ x, long long nr, T scale) {
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < nr; f += (long long)gridDim.x * blockDim.x)
    x[f] = w[f].re * scale;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_cp_cplx(const T* __restrict__ x, cx<T>* __restrict__ w, long long nr, T scale) {
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < nr; f += (long long)gridDim.x * blockDim.x)
    w[f] = {x[f] * scale, (T)0};
}

// the real parametrisation of the spectrum y, two coordinates per thread
// and round, into the epilogue (or written out); coordinates past nr are 0
template <typename T, class Epi>
__global__ void __launch_bounds__(256)
k_cp_unmap(const cx<T>* __restrict__ y, T* __restrict__ out, long long n, long long nr, int n1, int n2, int n3,
           Epi epi, const int* skip) {
  if (skip && *skip) return;
  const T sq2 = (T)1.41421356237309504880;
  constexpr int NQ = Epi::NRED > 0 ? Epi::NRED : 1;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n / 2;
       j += (long long)gridDim.x * blockDim.x) {
    T v[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const long long f = 2 * j + k;
      v[k] = (T)0;
      if (f < nr) {
        long long mf;
        const int c = cp_freq(f, n1, n2, n3, mf);
        const cx<T> h = y[f];
        v[k] = c == 0 ? h.re : (c == 1 ? sq2 * h.re : -sq2 * h.im);
      }
    }
    if constexpr (Epi::NRED > 0)
      epi(j, cx<T>{v[0], v[1]}, acc, false);
    else
      reinterpret_cast<cx<T>*>(out)[j] = {v[0], v[1]};
  }
  if constexpr (Epi::NRED > 0) {
    __shared__ double red[NQ * 4];
    block_sums_store<256, Epi::NRED, Epi::NMAX>(acc, epi.partial, epi.pstride, red);
  }
}

// one complex pass of the full-spectrum transforms: pencils of length L,
// geometry (inner, outer, element stride, count) as in StridedGeom; the
// strided pass without the m = 0 plane (axis-2 kernels) serves every axis
template <typename T, int DIR>
void cp_pass(int L, int inner, long long outer, long long estride, int batch, cx<T>* w, const cx<T>* tw,
             const int* skip, hipStream_t s) {
  if (L == 1) return;
  StridedGeom<T> geo;
  geo.inner = inner;
  geo.outer = outer;
  geo.estride = estride;
  geo.batch = batch;
  const int tm = pass_tm(int(sizeof(cx<T>)), L, 2, DIR);
  launch_axis12_L<T, 2, DIR>(L, dim3((batch + tm - 1) / tm), w, w, geo, tw, 1, 1, EpiNone{}, skip, s);
}

}  // namespace

// the workgroups of the pencil tiles alone (the launch adds those of the
// m = 0 plane in front of them on axis 1)
int axis12_tiles(const Grid& g, int axis, int elem_bytes, int dir) {
  const int L = axis == 1 ? g.n1 : g.n2;
  const int batch = axis == 1 ? g.n2 * g.m : g.n1 * g.m;
  const int tm = pass_tm(elem_bytes, L, axis, dir);
  return (batch + tm - 1) / tm;
}

int axis12_blocks(const Grid& g, int axis, int elem_bytes, int dir) {
  return axis12_tiles(g, axis, elem_bytes, dir) + (axis == 1 ? plane0_groups(dir) : 0);
}

bool fft_extent_supported(int N, int axis) {
  AnyPlan pl;
  if (N > kAnyMaxLen) return false;
  if (axis != 3) return N >= 1 && (templated12(N) || any_plan(N, pl));
  // an odd N3 takes full-length complex pencils, an even one half-length
  // pencils of the real transforms
  if (N % 2 == 1) return N >= 3 && (templated12(N) || any_plan(N, pl));
  return N >= 4 && (templated3(N / 2) || any_plan(N / 2, pl));
}

template <typename T>
void launch_axis12(const Grid& g, int axis, int dir, const T* src, T* dst, const Twiddles<T>& tw, int epi,
                   const EpiArgs<T>* ea, const int* skip, hipStream_t s) {
  const int L = axis == 1 ? g.n1 : g.n2;
  const cx<T>* twp = axis == 1 ? tw.t1 : tw.t2;
  StridedGeom<T> geo = geom<T>(g, axis);
  dim3 grid(axis12_tiles(g, axis, (int)sizeof(cx<T>), dir));
  const cx<T>* cs = reinterpret_cast<const cx<T>*>(src);
  cx<T>* cd = reinterpret_cast<cx<T>*>(dst);
  if (axis == 1) {
    if (dir > 0) {
      const bool up = ea && ea->k.u.zb;
      EpiP<T> pro{up ? reinterpret_cast<cx<T>*>(ea->k.u.pb) : nullptr,
                  up ? reinterpret_cast<const cx<T>*>(ea->k.u.zb) : nullptr, up ? ea->k.u.beta : nullptr};
      launch_axis12_L<T, 1, +1>(L, grid, cs, cd, geo, twp, g.m, g.n2, pro, skip, s);
    } else if (epi == EPI_K) {
      launch_axis12_L<T, 1, -1>(L, grid, cs, cd, geo, twp, g.m, g.n2, EpiK<T>{ea->k, ea->partial, ea->pstride}, skip,
                                s);
    } else if (epi == EPI_R) {
      if constexpr (std::is_same<T, double>::value)
        launch_axis12_L<T, 1, -1>(L, grid, cs, cd, geo, twp, g.m, g.n2, EpiR{ea->r, ea->partial, ea->pstride}, skip,
                                  s);
    } else {
      launch_axis12_L<T, 1, -1>(L, grid, cs, cd, geo, twp, g.m, g.n2, EpiNone{}, skip, s);
    }
  } else {
    if (dir > 0)
      launch_axis12_L<T, 2, +1>(L, grid, cs, cd, geo, twp, g.m, g.n2, EpiNone{}, skip, s);
    else
      launch_axis12_L<T, 2, -1>(L, grid, cs, cd, geo, twp, g.m, g.n2, EpiNone{}, skip, s);
  }
}

template <typename T>
void launch_axis3(const Grid& g, int mode, const T* src, T* dst, const uint32_t* maskbits, const Twiddles<T>& tw,
                  const int* skip, hipStream_t s) {
  const int L = g.m;
  const int np = g.n1 * g.n2;
  // the packing helpers leave sqrt2 (inverse input) and 2 (forward output;
  // DC and Nyquist 1) to these scales with the 1/sqrt(n) of each transform;
  // a full pass carries the inverse's factors into its forward output
  const double rn = 1.0 / std::sqrt((double)g.n), r2 = std::sqrt(2.0);
  const bool full = mode == A3_FULL;
  const T sc_c2r = (T)(rn / r2);
  const T sc_dc = (T)(full ? rn * rn / r2 : rn);
  const T sc_ac = (T)(full ? rn * rn / 2.0 : rn / r2);
  const cx<T>* cs = reinterpret_cast<const cx<T>*>(src);
  cx<T>* cd = reinterpret_cast<cx<T>*>(dst);
#define CSIPM_A3(LL)                                                                                      \
  case LL:                                                                                                \
    launch_axis3_at<T, LL>(mode, np, cs, cd, maskbits, tw.tm, tw.t3, sc_c2r, sc_dc, sc_ac, skip, s); \
    break;
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
      if (!launch_axis3_mixed<T>(L, mode, np, cs, cd, maskbits, tw.tm, tw.t3, sc_c2r, sc_dc, sc_ac, skip, s))
        (void)launch_axis3_any<T>(L, mode, np, cs, cd, maskbits, tw.tm, tw.t3, sc_c2r, sc_dc, sc_ac, skip, s);
      break;
  }
#undef CSIPM_A3
}

template <typename Te, typename Ti>
void launch_to_internal(const Grid& g, const Te* ext, Ti* in, hipStream_t s) {
  hipLaunchKernelGGL((k_to_internal<Te, Ti>), dim3(grid_for(g.n, 256)), dim3(256), 0, s, ext, in, g.n, g.nr, g.n1,
                     g.n2, g.n3, g.m);
}
template <typename Ti, typename Te>
void launch_to_external(const Grid& g, const Ti* in, Te* ext, hipStream_t s) {
  hipLaunchKernelGGL((k_to_external<Ti, Te>), dim3(grid_for(g.nr, 256)), dim3(256), 0, s, in, ext, g.nr, g.n1,
                     g.n2, g.n3, g.m);
}
void launch_feat_to_external(const Grid& g, const float* in, float* ext, hipStream_t s) {
  hipLaunchKernelGGL(k_feat_to_external, dim3(grid_for(g.nr, 256)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(in), reinterpret_cast<float4*>(ext), g.nr, g.n1, g.n2, g.n3,
                     g.m);
}
void launch_pack_mask(const Grid& g, const uint8_t* obs, uint32_t* bits, hipStream_t s) {
  const long long nw = (g.nr + 31) / 32;
  hipLaunchKernelGGL(k_pack_mask, dim3(grid_for(nw, 256)), dim3(256), 0, s, obs, bits, nw, g.nr);
}

// ------------------------------------------------ odd N3: full spectrum --
int cp_blocks(const Grid& g) {
  long long b = (g.n / 2 + 255) / 256;
  if (b > kCpMaxBlocks) b = kCpMaxBlocks;
  return (int)(b < 1 ? 1 : b);
}

template <typename T>
void cp_map(const Grid& g, const T* beta, T* work, const int* skip, hipStream_t s) {
  hipLaunchKernelGGL((k_cp_map<T>), dim3(grid_for(g.nr, 256)), dim3(256), 0, s, beta,
                     reinterpret_cast<cx<T>*>(work), g.nr, g.n1, g.n2, g.n3, skip);
}

template <typename T>
void cp_pupdate(const Grid& g, T* pb, T* pz, const T* zb, const T* zz, const double* beta, const int* skip,
                hipStream_t s) {
  hipLaunchKernelGGL((k_cp_pupd<T>), dim3(grid_for(g.n, 256)), dim3(256), 0, s, pb, pz, zb, zz, beta, g.n, skip);
}

template <typename T>
void cp_passes(const Grid& g, int dir, T* work, const Twiddles<T>& tw, const int* skip, hipStream_t s) {
  cx<T>* w = reinterpret_cast<cx<T>*>(work);
  const long long p3 = (long long)g.n2 * g.n3;
  if (dir > 0) {
    cp_pass<T, +1>(g.n1, (int)p3, 0, p3, (int)p3, w, tw.t1, skip, s);
    cp_pass<T, +1>(g.n2, g.n3, p3, g.n3, g.n1 * g.n3, w, tw.t2, skip, s);
    cp_pass<T, +1>(g.n3, 1, g.n3, 1, g.n1 * g.n2, w, tw.t3, skip, s);
  } else {
    cp_pass<T, -1>(g.n3, 1, g.n3, 1, g.n1 * g.n2, w, tw.t3, skip, s);
    cp_pass<T, -1>(g.n2, g.n3, p3, g.n3, g.n1 * g.n3, w, tw.t2, skip, s);
    cp_pass<T, -1>(g.n1, (int)p3, 0, p3, (int)p3, w, tw.t1, skip, s);
  }
}

template <typename T>
void cp_mask(const Grid& g, T* work, const uint32_t* bits, const int* skip, hipStream_t s) {
  hipLaunchKernelGGL((k_cp_mask<T>), dim3(grid_for(g.nr, 256)), dim3(256), 0, s, reinterpret_cast<cx<T>*>(work),
                     bits, g.nr, (T)(1.0 / (double)g.nr), skip);
}

template <typename T>
void cp_real(const Grid& g, const T* work, T* x, hipStream_t s) {
  hipLaunchKernelGGL((k_cp_real<T>), dim3(grid_for(g.nr, 256)), dim3(256), 0, s,
                     reinterpret_cast<const cx<T>*>(work), x, g.nr, (T)(1.0 / std::sqrt((double)g.nr)));
}

template <typename T>
void cp_cplx(const Grid& g, const T* x, T* work, hipStream_t s) {
  hipLaunchKernelGGL((k_cp_cplx<T>), dim3(grid_for(g.nr, 256)), dim3(256), 0, s, x, reinterpret_cast<cx<T>*>(work),
                     g.nr, (T)(1.0 / std::sqrt((double)g.nr)));
}

template <typename T>
int cp_unmap(const Grid& g, const T* work, T* out, int epi, const EpiArgs<T>* ea, const int* skip, hipStream_t s) {
  const cx<T>* y = reinterpret_cast<const cx<T>*>(work);
  const int nb = cp_blocks(g);
  if (epi == EPI_K) {
    KArgs<T> k = ea->k;
    k.u = PUpd<T>{};   // (the direction update ran before the map)
    hipLaunchKernelGGL((k_cp_unmap<T, EpiK<T>>), dim3(nb), dim3(256), 0, s, y, out, g.n, g.nr, g.n1, g.n2, g.n3,
                       EpiK<T>{k, ea->partial, ea->pstride}, skip);
  } else if (epi == EPI_R) {
    if constexpr (std::is_same<T, double>::value)
      hipLaunchKernelGGL((k_cp_unmap<T, EpiR>), dim3(nb), dim3(256), 0, s, y, out, g.n, g.nr, g.n1, g.n2, g.n3,
                         EpiR{ea->r, ea->partial, ea->pstride}, skip);
  } else {
    hipLaunchKernelGGL((k_cp_unmap<T, EpiNone>), dim3(nb), dim3(256), 0, s, y, out, g.n, g.nr, g.n1, g.n2, g.n3,
                       EpiNone{}, skip);
  }
  return nb;
}

#define CSIPM_CP_INST(T)                                                                                       \
  template void cp_map<T>(const Grid&, const T*, T*, const int*, hipStream_t);                                 \
  template void cp_pupdate<T>(const Grid&, T*, T*, const T*, const T*, const double*, const int*, hipStream_t); \
  template void cp_passes<T>(const Grid&, int, T*, const Twiddles<T>&, const int*, hipStream_t);               \
  template void cp_mask<T>(const Grid&, T*, const uint32_t*, const int*, hipStream_t);                         \
  template void cp_real<T>(const Grid&, const T*, T*, hipStream_t);                                            \
  template void cp_cplx<T>(const Grid&, const T*, T*, hipStream_t);                                            \
  template int cp_unmap<T>(const Grid&, const T*, T*, int, const EpiArgs<T>*, const int*, hipStream_t);
CSIPM_CP_INST(double)
CSIPM_CP_INST(float)
#undef CSIPM_CP_INST

#define CSIPM_INST(T)                                                                                          \
  template void launch_axis12<T>(const Grid&, int, int, const T*, T*, const Twiddles<T>&, int,                 \
                                 const EpiArgs<T>*, const int*, hipStream_t);                                  \
  template void launch_axis3<T>(const Grid&, int, const T*, T*, const uint32_t*, const Twiddles<T>&,           \
                                const int*, hipStream_t);                                                      \
  template void launch_to_internal<double, T>(const Grid&, const double*, T*, hipStream_t);                   \
  template void launch_to_internal<float, T>(const Grid&, const float*, T*, hipStream_t);                     \
  template void launch_to_external<T, double>(const Grid&, const T*, double*, hipStream_t);                   \
  template void launch_to_external<T, float>(const Grid&, const T*, float*, hipStream_t);
CSIPM_INST(double)
CSIPM_INST(float)
#undef CSIPM_INST

}  // namespace csipm
