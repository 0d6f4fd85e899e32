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
// factors.  Strided passes map consecutive lanes to consecutive pencils, so
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
      (void)launch_axis12_mixed<T, AX, DIR, Epi>(L, grid, src, dst, geo, tw, m, n2, epi, skip, s);
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

// the workgroups of the pencil tiles alone (the launch adds those of the
// m = 0 plane in front of them on axis 1)
int axis12_tiles(const Grid& g, int axis, int elem_bytes, int dir) {
  const int L = axis == 1 ? g.n1 : g.n2;
  const int batch = axis == 1 ? g.n2 * g.m : g.n1 * g.m;
  const int tm = strided_tm(elem_bytes, L, axis, dir);
  return (batch + tm - 1) / tm;
}

int axis12_blocks(const Grid& g, int axis, int elem_bytes, int dir) {
  return axis12_tiles(g, axis, elem_bytes, dir) + (axis == 1 ? plane0_groups(dir) : 0);
}

bool fft_extent_supported(int N, int axis) {
  if (axis != 3 && (N == 1 || N == 2)) return true;
#define CSIPM_IS_ODD(NN) if (axis != 3 && N == NN) return true;
  CSIPM_ODD_LENGTHS(CSIPM_IS_ODD)
#undef CSIPM_IS_ODD
  if (N >= 4 && N <= 1024 && (N & (N - 1)) == 0) return true;
#define CSIPM_IS(NN) if (N == NN) return true;
  CSIPM_MIXED_LENGTHS(CSIPM_IS)
#undef CSIPM_IS
  return false;
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
  const double rn = 1.0 / std::sqrt((double)g.n);
  const T sc_c2r = (T)rn;
  const T sc_dc = (T)rn;
  const T sc_ac = (T)(rn * std::sqrt(2.0));
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
      (void)launch_axis3_mixed<T>(L, mode, np, cs, cd, maskbits, tw.tm, tw.t3, sc_c2r, sc_dc, sc_ac, skip, s);
      break;
  }
#undef CSIPM_A3
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
  const long long nw = (g.n + 31) / 32;
  hipLaunchKernelGGL(k_pack_mask, dim3(grid_for(nw, 256)), dim3(256), 0, s, obs, bits, nw, g.n);
}

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
