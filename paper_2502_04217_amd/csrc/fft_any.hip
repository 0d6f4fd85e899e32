// Pencil passes at the grid extents 2^a 3^b 5^c 7^d up to 1024 that have no
// instantiated kernels (fft.hip and fft_mixed_f64/f32.hip instantiate the
// powers of two, the paper's non-power-of-two sizes and a few small ones).
// They compute what k_axis12 and k_axis3 compute — the m = 0 plane mixing,
// the fused direction update, the K and refinement epilogues, the axis-3
// c2r / mask / r2c — through the same helpers, but the pencils stay in LDS
// for the whole transform and its Stockham stages follow a radix plan
// computed at launch (radix 8, then one 4 or 2, for the power-of-two part;
// 3, 5 and 7 for the odd part), so that one kernel serves every length.
//
// A workgroup holds TM pencils (a power of two, TM L <= 4096 elements: at
// most 64 KB of FP64 tile) with NT = threads / TM threads each (512 threads
// of at most 8 elements in FP32, 256 of at most 16 in FP64), and the pencil
// length's twiddle table.  A
// stage loads every butterfly of the thread into registers, synchronises,
// and writes its outputs back in place.
#include "fft_kernels.h"

#include <algorithm>

namespace csipm {
namespace fftk {

namespace {

// threads per workgroup and elements per thread at most (TM L <= 4096):
// FP32 on 512 threads of at most 8 values, FP64 on 256 threads of at most
// 16 (each the faster of the two shapes measured in its precision)
template <typename T>
constexpr int any_threads() { return sizeof(T) == 4 ? 512 : 256; }
template <typename T>
constexpr int any_max_e() { return 4096 / any_threads<T>(); }

// Applies one radix-R stage (Ns: product of the earlier radices) to the
// pencil at a (element e at a[e * es]), in place; thread t of nt.
template <typename T, int R, int DIR>
__device__ __forceinline__ void any_stage(cx<T>* a, int es, int L, int Ns, int t, int nt,
                                          const cx<T>* __restrict__ tw) {
  constexpr int NB = (any_max_e<T>() + R - 1) / R;
  const int nbf = L / R;
  const int step = L / (Ns * R);
  cx<T> v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + i * nt;
    if (j < nbf) {
#pragma unroll
      for (int q = 0; q < R; ++q) v[i][q] = a[(j + q * nbf) * es];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + i * nt;
    if (j < nbf) {
      const int jm = j % Ns;
      if (Ns > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) v[i][q] = cmul(v[i][q], twiddle<T>(tw, jm * q * step, DIR));
      }
      dft_any<R, DIR, T>(v[i]);
      const int o = (j - jm) * R + jm;
#pragma unroll
      for (int q = 0; q < R; ++q) a[(o + q * Ns) * es] = v[i][q];
    }
  }
}

// The whole transform of the pencil at a; every thread of the workgroup
// calls it (it synchronises), and on return the result is in place and
// visible to all threads.
template <typename T, int DIR>
__device__ __forceinline__ void any_fft(cx<T>* a, int es, const AnyPlan& pl, int t, int nt,
                                        const cx<T>* __restrict__ tw) {
  int ns = 1;
  for (int s = 0; s < pl.nst; ++s) {
    const int r = pl.r[s];
    __syncthreads();
    switch (r) {
      case 8: any_stage<T, 8, DIR>(a, es, pl.L, ns, t, nt, tw); break;
      case 4: any_stage<T, 4, DIR>(a, es, pl.L, ns, t, nt, tw); break;
      case 2: any_stage<T, 2, DIR>(a, es, pl.L, ns, t, nt, tw); break;
      case 3: any_stage<T, 3, DIR>(a, es, pl.L, ns, t, nt, tw); break;
      case 5: any_stage<T, 5, DIR>(a, es, pl.L, ns, t, nt, tw); break;
      default: any_stage<T, 7, DIR>(a, es, pl.L, ns, t, nt, tw); break;
    }
    ns *= r;
  }
  __syncthreads();
}

// Strided pass (axis 1 or 2) of k_axis12 with the pencils in LDS: pencil p
// of the workgroup at element stride TM, then (axis 1) the partner rows of
// the m = 0 lanes.
template <typename T, int AX, int DIR, class Epi>
__global__ void __launch_bounds__(any_threads<T>())
k_axis12_any(const cx<T>* src, cx<T>* dst, StridedGeom<T> geo, const cx<T>* __restrict__ tw, int m, Plane0 pl,
             Epi epi, const int* skip, AnyPlan plan, int TM, int rows) {
  if (skip && *skip) return;
  constexpr bool MIX = AX == 1;
  const int L = plan.L;
  const int NT = any_threads<T>() / TM;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tile = reinterpret_cast<cx<T>*>(smem_raw);
  const int p = threadIdx.x % TM;
  const int t = threadIdx.x / TM;
  const Lane12 ln = lane12<AX, DIR>(p, TM, geo, m, pl);
  cx<T>* a = tile + p;
  // the twiddle table, after the tile and the partner rows (the stages read
  // it after their first barrier)
  cx<T>* twl = tile + (size_t)rows * L;
  for (int i = threadIdx.x; i < L; i += any_threads<T>()) twl[i] = tw[i];

  bool upd = false;
  T be = T(0);
  if constexpr (Epi::PRO) {
    upd = epi.z != nullptr;
    if (upd) be = (T)*epi.beta;
  }
  for (int e = t; e < L; e += NT)
    a[e * TM] = load_input(src, ln.base + (long long)e * geo.estride, ln.active, upd, be, epi, MIX && ln.m0);
  if constexpr (MIX) {
    cx<T>* stg = tile + TM * L;
    int slot;
    if (stage_partners<T, DIR>(stg, src, L, TM, any_threads<T>(), geo, m, pl, epi, upd, be, ln.ded, p, slot) > 0 &&
        ln.m0 && ln.active) {
      for (int e = t; e < L; e += NT) a[e * TM] = plane0_mix<T, DIR>(a[e * TM], stg[slot * L + e], e, ln, L, pl.n2);
    }
  }
  any_fft<T, DIR>(a, TM, plan, t, NT, twl);

  if constexpr (Epi::NRED > 0) {
    double acc[Epi::NRED];
#pragma unroll
    for (int q = 0; q < Epi::NRED; ++q) acc[q] = 0.0;
    if (ln.active) {
      for (int e = t; e < L; e += NT) {
        cx<T> h = a[e * TM];
        if (plane0_keep<AX, DIR>(e, h, ln, L, pl.n2)) epi(ln.base + (long long)e * geo.estride, h, acc, MIX && ln.m0);
      }
    }
    block_sums_store<any_threads<T>(), Epi::NRED, Epi::NMAX>(acc, epi.partial, epi.pstride,
                                                       reinterpret_cast<double*>(smem_raw));
  } else {
    if (ln.active) {
      for (int e = t; e < L; e += NT) {
        cx<T> h = a[e * TM];
        if (plane0_keep<AX, DIR>(e, h, ln, L, pl.n2)) dst[ln.base + (long long)e * geo.estride] = h;
      }
    }
  }
}

// Axis-3 pass of k_axis3 (half length L = N3/2, contiguous pencils) with the
// pencils in LDS.  The transform work uses the strided passes' tile layout,
// element e of pencil p at e (TM + 1) + p with the pencils in consecutive
// lanes, on which every stage access is free of bank conflicts (a tile of
// whole pencils conflicts on the strided Stockham writes); the workgroup's TM
// pencils, one contiguous run of TM L values in memory, are loaded and stored
// through the same tile with consecutive lanes on consecutive values.
template <typename T, int MODE>
__global__ void __launch_bounds__(any_threads<T>())
k_axis3_any(const cx<T>* src, cx<T>* dst, const uint32_t* __restrict__ mask, const cx<T>* __restrict__ twm,
            const cx<T>* __restrict__ tw3, int npencils, T sc_c2r, T sc_r2c_dc, T sc_r2c, const int* skip,
            AnyPlan plan, int TM) {
  if (skip && *skip) return;
  constexpr int NTHR = any_threads<T>();
  constexpr int EM = any_max_e<T>();
  const int L = plan.L;
  const int NT = NTHR / TM;
  const int N3 = 2 * L;
  const int ES = TM + 1;   // element row stride
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tile = reinterpret_cast<cx<T>*>(smem_raw);
  const int p = threadIdx.x % TM;
  const int t = threadIdx.x / TM;
  const int pen = blockIdx.x * TM + p;
  const bool active = pen < npencils;
  cx<T>* a = tile + p;
  // the half-length transform's twiddles, after the tile
  cx<T>* twl = tile + (size_t)L * ES;
  for (int i = threadIdx.x; i < L; i += NTHR) twl[i] = twm[i];
  // the workgroup's pencils: values [run, run + nval) of the array
  const long long run = (long long)blockIdx.x * TM * L;
  const int nval = min(TM, npencils - (int)blockIdx.x * TM) * L;
  for (int i = threadIdx.x; i < TM * L; i += NTHR) {
    const int pp = i / L, e = i - pp * L;
    tile[e * ES + pp] = i < nval ? src[run + i] : cx<T>{T(0), T(0)};
  }
  __syncthreads();
  if constexpr ((MODE & A3_C2R) != 0) {
    // Z_e needs X_e and X_{L-e}: all of X is read before any Z is written
    cx<T> z[EM];
#pragma unroll
    for (int i = 0; i < EM; ++i) {
      const int e = t + i * NT;
      if (e < L) z[i] = e == 0 ? c2r_dc(a[0]) : c2r_pack(a[e * ES], a[(L - e) * ES], tw3[e]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EM; ++i) {
      const int e = t + i * NT;
      if (e < L) a[e * ES] = z[i];
    }
    any_fft<T, +1>(a, ES, plan, t, NT, twl);
    for (int e = t; e < L; e += NT) {
      if constexpr (MODE == A3_FULL) {
        const long long bit = (long long)pen * N3 + 2 * e;
        a[e * ES] = mask_pair(a[e * ES], active ? mask[bit >> 5] : 0u, (int)(bit & 31));
      } else {
        a[e * ES] = cscale(a[e * ES], sc_c2r);
      }
    }
    if constexpr (MODE == A3_C2R) {
      __syncthreads();
      for (int i = threadIdx.x; i < nval; i += NTHR) {
        const int pp = i / L, e = i - pp * L;
        dst[run + i] = tile[e * ES + pp];
      }
      return;
    }
  }
  any_fft<T, -1>(a, ES, plan, t, NT, twl);
  {
    // X_e needs Z_e and Z_{L-e}: all of Z is read before any X is written
    cx<T> x[EM];
#pragma unroll
    for (int i = 0; i < EM; ++i) {
      const int e = t + i * NT;
      if (e < L) x[i] = e == 0 ? r2c_dc(a[0], sc_r2c_dc) : r2c_unpack(a[e * ES], a[(L - e) * ES], tw3[e], sc_r2c);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EM; ++i) {
      const int e = t + i * NT;
      if (e < L) a[e * ES] = x[i];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nval; i += NTHR) {
    const int pp = i / L, e = i - pp * L;
    dst[run + i] = tile[e * ES + pp];
  }
}

}  // namespace

bool any_plan(int L, AnyPlan& pl) {
  if (L < 1 || L > kAnyMaxLen) return false;
  int r = L, a = 0;
  while (r % 2 == 0) { r /= 2; ++a; }
  pl.L = L;
  pl.nst = 0;
  for (; a >= 3; a -= 3) pl.r[pl.nst++] = 8;
  if (a > 0) pl.r[pl.nst++] = 1 << a;
  for (int f : {3, 5, 7})
    while (r % f == 0) {
      r /= f;
      pl.r[pl.nst++] = f;
    }
  return r == 1;
}

int any_tm(int w, int L) {
  int tm = w == (int)sizeof(cx<float>) ? any_threads<float>() : any_threads<double>();
  while (tm > 1 && tm * L > 4096) tm >>= 1;
  return tm;
}

template <typename T, int AX, int DIR, class Epi>
bool launch_axis12_any(int L, dim3 grid, const cx<T>* src, cx<T>* dst, StridedGeom<T> geo, const cx<T>* tw, int m,
                       int n2, Epi epi, const int* skip, hipStream_t s) {
  AnyPlan plan;
  if (!any_plan(L, plan)) return false;
  const int tm = any_tm((int)sizeof(cx<T>), L);
  const Plane0 pl{n2, AX == 1 ? plane0_groups(DIR) : 0};
  // the tile, and on axis 1 the partner-row slots (at most 4 in the
  // first workgroup of the forward pass, (TM - 1) / m + 1 in a tile)
  const int rows = tm + (AX == 1 ? std::max(4, (tm - 1) / m + 1) : 0);
  const size_t shm = (size_t)(rows + 1) * L * sizeof(cx<T>);   // (and the twiddles)
  auto kern = k_axis12_any<T, AX, DIR, Epi>;
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL(kern, dim3(grid.x + pl.ndedicated), dim3(any_threads<T>()), shm, s, src, dst, geo, tw, m, pl, epi,
                     skip, plan, tm, rows);
  return true;
}

template <typename T>
bool launch_axis3_any(int L, int mode, int np, const cx<T>* cs, cx<T>* cd, const uint32_t* maskbits,
                      const cx<T>* twm, const cx<T>* tw3, T sc_c2r, T sc_dc, T sc_ac, const int* skip,
                      hipStream_t s) {
  AnyPlan plan;
  if (!any_plan(L, plan)) return false;
  const int tm = any_tm((int)sizeof(cx<T>), L);
  const size_t shm = ((size_t)L * (tm + 1) + L) * sizeof(cx<T>);   // (the tile and the twiddles)
  const dim3 grid((np + tm - 1) / tm), block(any_threads<T>());
  if (shm > 65536) {
    (void)hipFuncSetAttribute((const void*)k_axis3_any<T, A3_FULL>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    (void)hipFuncSetAttribute((const void*)k_axis3_any<T, A3_C2R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    (void)hipFuncSetAttribute((const void*)k_axis3_any<T, A3_R2C>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  }
  if (mode == A3_FULL)
    hipLaunchKernelGGL((k_axis3_any<T, A3_FULL>), grid, block, shm, s, cs, cd, maskbits, twm, tw3, np, sc_c2r, sc_dc,
                       sc_ac, skip, plan, tm);
  else if (mode == A3_C2R)
    hipLaunchKernelGGL((k_axis3_any<T, A3_C2R>), grid, block, shm, s, cs, cd, maskbits, twm, tw3, np, sc_c2r, sc_dc,
                       sc_ac, skip, plan, tm);
  else
    hipLaunchKernelGGL((k_axis3_any<T, A3_R2C>), grid, block, shm, s, cs, cd, maskbits, twm, tw3, np, sc_c2r, sc_dc,
                       sc_ac, skip, plan, tm);
  return true;
}

#define CSIPM_ANY12(T, AX, DIR, EPI)                                                                       \
  template bool launch_axis12_any<T, AX, DIR, EPI>(int, dim3, const cx<T>*, cx<T>*, StridedGeom<T>,        \
                                                   const cx<T>*, int, int, EPI, const int*, hipStream_t);
#define CSIPM_ANY(T)                                                                                        \
  CSIPM_ANY12(T, 1, +1, EpiP<T>)                                                                            \
  CSIPM_ANY12(T, 1, -1, EpiNone)                                                                            \
  CSIPM_ANY12(T, 1, -1, EpiK<T>)                                                                            \
  CSIPM_ANY12(T, 2, +1, EpiNone)                                                                            \
  CSIPM_ANY12(T, 2, -1, EpiNone)                                                                            \
  template bool launch_axis3_any<T>(int, int, int, const cx<T>*, cx<T>*, const uint32_t*, const cx<T>*,     \
                                    const cx<T>*, T, T, T, const int*, hipStream_t);
CSIPM_ANY(double)
CSIPM_ANY(float)
CSIPM_ANY12(double, 1, -1, EpiR)
#undef CSIPM_ANY
#undef CSIPM_ANY12

}  // namespace fftk
}  // namespace csipm
