// C-ABI of the csipm library: problem set-up, the interior-point driver, the
// Krylov drivers and single-operator applies.  Host code; all arithmetic on
// the vectors happens in the kernels of fft.hip, vec.hip and mlp.hip.
#include "../../include/csipm.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "csipm_internal.h"
#include "mlp.h"
#include "vec.h"

using namespace csipm;

namespace {

constexpr size_t kAlign = 256;


struct Carver {
  char* base;
  size_t off = 0;
  size_t cap;
  template <typename T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += count * sizeof(T);
    return p;
  }
};

}  // namespace

struct csipm_ctx {
  Grid g{};
  hipStream_t s = nullptr;
  int device = 0;       // the HIP device current at creation
  std::string err;

  // FP64 interior-point state and Newton system (internal layout); hb
  // holds G = H beta - xi, the data part of the first KKT row
  double *beta, *z, *nu1, *nu2, *xi, *hb, *sig1, *sig2, *rhb, *rhz, *dxb, *dxz, *diagH;
  // copy of (beta, z, nu1, nu2) taken before a step along a direction that
  // missed its tolerance, restored if that step raised rel_kkt
  double *snap;
  // FP64 Krylov vectors and FFT work array
  double *rb, *rz, *zb, *zz, *pb, *pz, *qb, *qz, *work;
  // FP32 Krylov set
  float *sig1f, *sig2f, *frb, *frz, *fzb, *fzz, *fpb, *fpz, *fqb, *fqz, *fxb, *fxz, *fwork;
  float *fwb, *fwz;   // FP32 w = K z of conjugate residuals
  double *yb64, *yz64; // CAr: y = P^{-1} K v (FP64)
  double *dab, *daz;   // predictor-corrector: the affine direction
  float *fyb, *fyz;    // CAr: y (FP32)
  // learned correction
  float *pc_c, *feat, *mlp_params;
  // per 64-coefficient chunk: the correction's gate passes somewhere in the
  // last updated iterate (written by the update), and c may differ from 1
  // there (pc_set; valid while pc_tracked: otherwise c may differ anywhere)
  uint32_t *pc_act, *pc_set;
  bool pc_tracked = false;
  uint32_t* mask;
  cx<double>* tw64;
  cx<float>* tw32;
  Twiddles<double> T64;
  Twiddles<float> T32;
  double *partK, *partV, *scal;
  int* flags;
  // host side
  double* hscal = nullptr;   // pinned: S_COUNT doubles then F_COUNT ints
  int* hflags = nullptr;
  double lambda = 0.0;
  bool have_lambda = false;
  bool have_params = false;
  double xi_inf = 0.0;
  long long nobs = 0;
  double setup_s = 0.0;   // wall time of csipm_create
  std::vector<csipm_iter_log> log;
  // capture of training records
  int cap_enable = 0, cap_per_iter = 0, cap_max = 0, cap_count = 0;
  float *cap_feat = nullptr, *cap_rec = nullptr;
  unsigned long long cap_seed = 0;
  std::vector<int> cap_cg;
  // iterations of the last PCG solve: the first chunk of the next one
  int pcg_hint = 0;
  // kernel timing: an event pair per launch while kt_on
  bool kt_on = false;
  std::vector<hipEvent_t> kt_ev;
  std::vector<std::pair<const char*, size_t>> kt_rec;
  long long kt_dropped = 0;
  // PCG chunks recorded as HIP graphs (pcg), keyed by precision, chunk
  // length, whether the chunk starts the solve, and the correction pointer;
  // recorded on a private stream, replayed on s
  struct PcgGraph {
    int wbytes, chunk;
    bool first;
    const float* pcc;
    hipGraphExec_t exec;
  };
  std::vector<PcgGraph> graphs;
  hipStream_t cap_s = nullptr;
  long long solves = 0;   // csipm_solve calls that returned (graphs from the second on)
};

namespace {

csipm_status fail(csipm_ctx* c, csipm_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

csipm_status hip_check(csipm_ctx* c, const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, CSIPM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
  return CSIPM_OK;
}

// Kernel timing.  KT(c, name, launch) brackets one launcher call with a pair
// of events on the context's stream when timing is enabled.
constexpr size_t kMaxTimed = 1000000;

size_t kt_begin(csipm_ctx* c, const char* name) {
  if (!c->kt_on) return SIZE_MAX;
  if (c->kt_rec.size() >= kMaxTimed) {
    ++c->kt_dropped;
    return SIZE_MAX;
  }
  const size_t e = 2 * c->kt_rec.size();
  while (c->kt_ev.size() < e + 2) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) {
      ++c->kt_dropped;
      return SIZE_MAX;
    }
    c->kt_ev.push_back(ev);
  }
  (void)hipEventRecord(c->kt_ev[e], c->s);
  c->kt_rec.emplace_back(name, e);
  return e;
}
void kt_end(csipm_ctx* c, size_t e) {
  if (e != SIZE_MAX) (void)hipEventRecord(c->kt_ev[e + 1], c->s);
}
#define KT(c, name, launch)                 \
  do {                                      \
    const size_t kt_e_ = kt_begin(c, name); \
    launch;                                 \
    kt_end(c, kt_e_);                       \
  } while (0)
// kernel name with the precision of T
#define PN(T, s) (sizeof(T) == 8 ? s ".f64" : s ".f32")

// Copies the device scalar and flag blocks to pinned host memory and waits.
csipm_status sync_scalars(csipm_ctx* c, const char* where) {
  hipError_t e = hipMemcpyAsync(c->hscal, c->scal, sizeof(double) * S_COUNT, hipMemcpyDeviceToHost, c->s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->hflags, c->flags, sizeof(int) * F_COUNT, hipMemcpyDeviceToHost, c->s);
  if (e == hipSuccess) e = hipStreamSynchronize(c->s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fail(c, CSIPM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
  return CSIPM_OK;
}

// partial sums of one K-apply: one per workgroup of the axis-1 forward pass
// (of the unmap pass for an odd N3)
size_t k_partials(int n1, int n2, int n3) {
  const Grid g = make_grid(n1, n2, n3);
  if (g.odd3()) return (size_t)cp_blocks(g) + 64;
  return (size_t)std::max(axis12_blocks(g, 1, 16, -1), axis12_blocks(g, 1, 8, -1)) + 64;
}

size_t layout(Carver& cv, csipm_ctx* c, int n1, int n2, int n3) {
  const Grid g = make_grid(n1, n2, n3);
  const size_t n = (size_t)g.n;
  // FFT scratch: the half spectrum (n reals), or the whole spectrum for an odd N3
  const size_t nw = g.odd3() ? std::max(n, (size_t)(2 * g.nr)) : n;
  const size_t ntw = (size_t)n1 + n2 + n3 / 2 + n3;
  double** d64[] = {&c->beta, &c->z, &c->nu1, &c->nu2, &c->xi, &c->hb, &c->sig1, &c->sig2, &c->rhb, &c->rhz,
                    &c->dxb, &c->dxz, &c->diagH, &c->rb, &c->rz, &c->zb, &c->zz, &c->pb, &c->pz, &c->qb,
                    &c->qz, &c->yb64, &c->yz64, &c->dab, &c->daz};
  for (double** p : d64) *p = cv.take<double>(n);
  c->work = cv.take<double>(nw);
  c->snap = cv.take<double>(4 * n);
  float** f32[] = {&c->sig1f, &c->sig2f, &c->frb, &c->frz, &c->fzb, &c->fzz, &c->fpb, &c->fpz, &c->fqb,
                   &c->fqz,   &c->fxb,   &c->fxz, &c->pc_c, &c->fwb, &c->fwz, &c->fyb, &c->fyz};
  for (float** p : f32) *p = cv.take<float>(n);
  c->fwork = cv.take<float>(nw);
  c->feat = cv.take<float>(4 * n);
  c->mlp_params = cv.take<float>(CSIPM_MLP_PARAMS);
  c->mask = cv.take<uint32_t>((n + 31) / 32);
  c->pc_act = cv.take<uint32_t>((n + kPcChunk - 1) / kPcChunk);
  c->pc_set = cv.take<uint32_t>((n + kPcChunk - 1) / kPcChunk);
  c->tw64 = cv.take<cx<double>>(ntw);
  c->tw32 = cv.take<cx<float>>(ntw);
  c->partK = cv.take<double>(2 * k_partials(n1, n2, n3));   // up to two quantities
  c->partV = cv.take<double>((size_t)VEC_MAX_BLOCKS * 16);
  c->scal = cv.take<double>(S_COUNT);
  c->flags = cv.take<int>(F_COUNT);
  return cv.off + kAlign;
}

// ------------------------------------------------------------- operators --
template <typename T>
const Twiddles<T>& tw(csipm_ctx* c);
template <>
const Twiddles<double>& tw<double>(csipm_ctx* c) { return c->T64; }
template <>
const Twiddles<float>& tw<float>(csipm_ctx* c) { return c->T32; }

// out = H in (internal layout), work = FFT scratch; out may not equal in
// (the axis-1 inverse pass reads the mirror rows of the m = 0 plane).
template <typename T>
void op_H(csipm_ctx* c, const T* in, T* out, T* work) {
  const Grid& g = c->g;
  if (g.odd3()) {
    KT(c, PN(T, "cp_map"), cp_map<T>(g, in, work, nullptr, c->s));
    KT(c, PN(T, "cp_inv"), cp_passes<T>(g, +1, work, tw<T>(c), nullptr, c->s));
    KT(c, PN(T, "cp_mask"), cp_mask<T>(g, work, c->mask, nullptr, c->s));
    KT(c, PN(T, "cp_fwd"), cp_passes<T>(g, -1, work, tw<T>(c), nullptr, c->s));
    KT(c, PN(T, "cp_unmap"), cp_unmap<T>(g, work, out, EPI_NONE, nullptr, nullptr, c->s));
    return;
  }
  KT(c, PN(T, "axis1_inv"), launch_axis12<T>(g, 1, +1, in, work, tw<T>(c), EPI_NONE, nullptr, nullptr, c->s));
  KT(c, PN(T, "axis2_inv"), launch_axis12<T>(g, 2, +1, work, work, tw<T>(c), EPI_NONE, nullptr, nullptr, c->s));
  KT(c, PN(T, "axis3"), launch_axis3<T>(g, A3_FULL, work, work, c->mask, tw<T>(c), nullptr, c->s));
  KT(c, PN(T, "axis2_fwd"), launch_axis12<T>(g, 2, -1, work, work, tw<T>(c), EPI_NONE, nullptr, nullptr, c->s));
  KT(c, PN(T, "axis1_fwd"), launch_axis12<T>(g, 1, -1, work, out, tw<T>(c), EPI_NONE, nullptr, nullptr, c->s));
}

// x = A in (real grid, row-major), work = FFT scratch (must differ from x).
template <typename T>
void op_A(csipm_ctx* c, const T* in, T* x, T* work) {
  const Grid& g = c->g;
  if (g.odd3()) {
    cp_map<T>(g, in, work, nullptr, c->s);
    cp_passes<T>(g, +1, work, tw<T>(c), nullptr, c->s);
    cp_real<T>(g, work, x, c->s);
    return;
  }
  launch_axis12<T>(g, 1, +1, in, work, tw<T>(c), EPI_NONE, nullptr, nullptr, c->s);
  launch_axis12<T>(g, 2, +1, work, work, tw<T>(c), EPI_NONE, nullptr, nullptr, c->s);
  launch_axis3<T>(g, A3_C2R, work, x, nullptr, tw<T>(c), nullptr, c->s);
}

// out = A^T x (internal layout).
template <typename T>
void op_At(csipm_ctx* c, const T* x, T* out, T* work) {
  const Grid& g = c->g;
  if (g.odd3()) {
    cp_cplx<T>(g, x, work, c->s);
    cp_passes<T>(g, -1, work, tw<T>(c), nullptr, c->s);
    (void)cp_unmap<T>(g, work, out, EPI_NONE, nullptr, nullptr, c->s);
    return;
  }
  launch_axis3<T>(g, A3_R2C, x, work, nullptr, tw<T>(c), nullptr, c->s);
  launch_axis12<T>(g, 2, -1, work, work, tw<T>(c), EPI_NONE, nullptr, nullptr, c->s);
  launch_axis12<T>(g, 1, -1, work, out, tw<T>(c), EPI_NONE, nullptr, nullptr, c->s);
}

size_t k_partials(int n1, int n2, int n3);

// q = K p with p.q partials in c->partK; returns the number of partials.
template <typename T>
int op_K(csipm_ctx* c, const T* pb, const T* pz, const T* s1, const T* s2, T* qb, T* qz, T* work,
         const int* skip, const PUpd<T>* u = nullptr) {
  const Grid& g = c->g;
  const int ps = (int)k_partials(g.n1, g.n2, g.n3);
  EpiArgs<T> ka{KArgs<T>{pb, pz, s1, s2, qb, qz, u ? *u : PUpd<T>{}}, RArgs{}, c->partK, ps};
  if (g.odd3()) {
    if (u)
      KT(c, PN(T, "cp_pupd"),
         cp_pupdate<T>(g, u->pb, u->pz, u->zb, u->zz, u->beta, skip, c->s));
    KT(c, PN(T, "cp_map"), cp_map<T>(g, pb, work, skip, c->s));
    KT(c, PN(T, "cp_inv"), cp_passes<T>(g, +1, work, tw<T>(c), skip, c->s));
    KT(c, PN(T, "cp_mask"), cp_mask<T>(g, work, c->mask, skip, c->s));
    KT(c, PN(T, "cp_fwd"), cp_passes<T>(g, -1, work, tw<T>(c), skip, c->s));
    int nb = 0;
    KT(c, PN(T, "cp_unmap_K"), nb = cp_unmap<T>(g, work, nullptr, EPI_K, &ka, skip, c->s));
    return nb;
  }
  const int nb5 = axis12_blocks(g, 1, (int)sizeof(cx<T>), -1);
  // (the passes that apply the direction update are timed under their own names)
  KT(c, u ? PN(T, "axis1_inv_P") : PN(T, "axis1_inv"),
     launch_axis12<T>(g, 1, +1, pb, work, tw<T>(c), EPI_NONE, u ? &ka : nullptr, skip, c->s));
  KT(c, PN(T, "axis2_inv"), launch_axis12<T>(g, 2, +1, work, work, tw<T>(c), EPI_NONE, nullptr, skip, c->s));
  KT(c, PN(T, "axis3"), launch_axis3<T>(g, A3_FULL, work, work, c->mask, tw<T>(c), skip, c->s));
  KT(c, PN(T, "axis2_fwd"), launch_axis12<T>(g, 2, -1, work, work, tw<T>(c), EPI_NONE, nullptr, skip, c->s));
  KT(c, u ? PN(T, "axis1_fwd_KP") : PN(T, "axis1_fwd_K"),
     launch_axis12<T>(g, 1, -1, work, work, tw<T>(c), EPI_K, &ka, skip, c->s));
  return nb5;
}

// FP64 refinement residual r = h - K d, fused into the K-apply of d: writes
// H d_beta (into rb), sums r.P_c^{-1}r -> scal[S_REF] and max |r| ->
// scal[S_REFINF].
void op_Kr(csipm_ctx* c, const float* pcc) {
  const Grid& g = c->g;
  const int ps = (int)k_partials(g.n1, g.n2, g.n3);
  // H d_beta goes to rb: the FP64 Krylov vectors are idle in the FP32 form
  RArgs ra{c->dxb, c->dxz, c->sig1, c->sig2, c->rhb, c->rhz, pcc, c->rb};
  EpiArgs<double> ea{KArgs<double>{}, ra, c->partK, ps};
  double* work = c->work;
  if (g.odd3()) {
    int nb = 0;
    KT(c, "cp_map.f64", cp_map<double>(g, c->dxb, work, nullptr, c->s));
    KT(c, "cp_inv.f64", cp_passes<double>(g, +1, work, c->T64, nullptr, c->s));
    KT(c, "cp_mask.f64", cp_mask<double>(g, work, c->mask, nullptr, c->s));
    KT(c, "cp_fwd.f64", cp_passes<double>(g, -1, work, c->T64, nullptr, c->s));
    KT(c, "cp_unmap_R.f64", nb = cp_unmap<double>(g, work, nullptr, EPI_R, &ea, nullptr, c->s));
    KT(c, "fin_sum", fin_sum(c->partK, nb, c->scal + S_REF, c->s));
    KT(c, "fin_max", fin_max(c->partK + ps, nb, c->scal + S_REFINF, c->s));
    return;
  }
  const int nb5 = axis12_blocks(g, 1, 16, -1);
  KT(c, "axis1_inv.f64", launch_axis12<double>(g, 1, +1, c->dxb, work, c->T64, EPI_NONE, nullptr, nullptr, c->s));
  KT(c, "axis2_inv.f64", launch_axis12<double>(g, 2, +1, work, work, c->T64, EPI_NONE, nullptr, nullptr, c->s));
  KT(c, "axis3.f64", launch_axis3<double>(g, A3_FULL, work, work, c->mask, c->T64, nullptr, c->s));
  KT(c, "axis2_fwd.f64", launch_axis12<double>(g, 2, -1, work, work, c->T64, EPI_NONE, nullptr, nullptr, c->s));
  KT(c, "axis1_fwd_R.f64", launch_axis12<double>(g, 1, -1, work, work, c->T64, EPI_R, &ea, nullptr, c->s));
  KT(c, "fin_sum", fin_sum(c->partK, nb5, c->scal + S_REF, c->s));
  KT(c, "fin_max", fin_max(c->partK + ps, nb5, c->scal + S_REFINF, c->s));
}

// ------------------------------------------------- learned correction --
// Features of the current iterate into c->feat (internal order) from the
// FP64 barrier diagonals in sig1/sig2 and max|beta| of the last residual.
void compute_features(csipm_ctx* c) {
  const long long n = c->g.n;
  mlp_mean_log_l1(c->sig1, c->sig2, n, c->partV, c->scal + S_MISC + 1, c->s);
  mlp_features(c->sig1, c->sig2, c->beta, c->diagH, c->scal + S_MISC + 1, c->scal + S_RESID + 4, c->feat, n, c->s);
}

// c = softplus(MLP(features)) + 1e-6 where it can act on P_c^{-1}, c = 1
// elsewhere; features formed from the interior-point state (before the
// Newton system is built).  With have_logsum the centring sum of log(S1+S2)
// is already in scal[S_RESID + 7] (reduced with the residual of this
// iterate); otherwise it is computed here.
csipm_status learned_correction(csipm_ctx* c, bool have_logsum) {
  const double* ml = c->scal + S_RESID + 7;
  double mscale = 1.0 / (double)c->g.n;
  if (!have_logsum) {
    KT(c, "log_l1+fin",
       mlp_mean_log_l1_state(c->beta, c->z, c->nu1, c->nu2, c->g.n, c->partV, c->scal + S_MISC + 1, c->s));
    ml = c->scal + S_MISC + 1;
    mscale = 1.0;
  }
  KT(c, "correction",
     mlp_correction_state(c->beta, c->z, c->nu1, c->nu2, c->diagH, ml, mscale, c->scal + S_RESID + 4, c->mlp_params,
                          c->pc_c, c->g.n, c->pc_set, c->s));
  c->pc_tracked = true;
  return hip_check(c, "learned_correction");
}

template <typename T>
void capture_pair(csipm_ctx* c, const T* pb, const T* pz, const T* qb, const T* qz, const T* s1, const T* s2) {
  compute_features(c);
  const size_t off = (size_t)c->cap_count * c->cap_per_iter;
  // policy capture draws among the coefficients where the correction acts;
  // their list goes to fwb (an FP32 n-array only the CR and CAr solvers use)
  mlp_capture<T>(pb, pz, qb, qz, s1, s2, c->feat, c->g.n, c->cap_per_iter,
                 c->cap_seed + (unsigned long long)c->cap_count * (unsigned long long)c->cap_per_iter,
                 c->cap_feat + off * 4, c->cap_rec + off * MLP_REC, c->partV,
                 c->cap_enable == 2 ? reinterpret_cast<int*>(c->fwb) : nullptr, kPcRelevance, c->s);
}

// ------------------------------------------------------------------- PCG --
struct PcgSet {
  void *rb, *rz, *zb, *zz, *pb, *pz, *qb, *qz, *work, *wb, *wz, *yb, *yz;
};

template <typename T>
PcgSet pcg_set(csipm_ctx* c);
template <>
PcgSet pcg_set<double>(csipm_ctx* c) {
  // w of conjugate residuals: the FP64 right-hand side copy is idle in the FP64 form
  return {c->rb, c->rz, c->zb, c->zz, c->pb, c->pz, c->qb, c->qz, c->work, c->rhb, c->rhz, c->yb64, c->yz64};
}
template <>
PcgSet pcg_set<float>(csipm_ctx* c) {
  return {c->frb, c->frz, c->fzb, c->fzz, c->fpb, c->fpz, c->fqb, c->fqz, c->fwork, c->fwb, c->fwz, c->fyb, c->fyz};
}

struct PcgOut {
  int iters = 0;
  bool converged = false;
  bool breakdown = false;
  double res0 = 0.0, res = 0.0;
};

// Preconditioned CG (Hestenes-Stiefel) on K x = h, x0 = 0, stopping on
// sqrt(r.P^{-1}r) <= max(atol, eta sqrt(r0.P^{-1}r0)).  The caller has put
// r = h and p = P^{-1}r into the precision-T Krylov vectors and finalised
// the start (k_fin_cg_init).  x0 = 0 is never stored: the first update
// writes x = alpha p.  On return r holds the recursive residual of x.
//
// One chunk of PCG iterations queued on c->s: K-apply of p (with the fused
// direction update after the solve's first iteration), alpha, the update of
// x, r, z and beta.  Finished iterations turn the rest of a chunk into
// no-ops through the device flag, so the host only synchronises once per
// chunk.  If `capture` is set, p_0 and q_0 = K p_0 go to the capture hook.
template <typename T>
void pcg_chunk(csipm_ctx* c, int chunk, bool first, T* xb, T* xz, const T* s1, const T* s2, const float* pcc,
               bool capture) {
  const long long n = c->g.n;
  PcgSet v = pcg_set<T>(c);
  T *rb = (T*)v.rb, *rz = (T*)v.rz, *zb = (T*)v.zb, *zz = (T*)v.zz, *pb = (T*)v.pb, *pz = (T*)v.pz,
    *qb = (T*)v.qb, *qz = (T*)v.qz, *work = (T*)v.work;
  const int nbv = vec_blocks(n);
  const int* skip = c->flags + F_DONE;
  // after the first iteration, p <- z + beta p is applied by the K-apply of
  // the new p as it reads p (PUpd), not by a separate pass
  const PUpd<T> upd{pb, pz, zb, zz, c->scal + S_BETA};
  for (int k = 0; k < chunk; ++k) {
    const int nbk = op_K<T>(c, pb, pz, s1, s2, qb, qz, work, skip, first ? nullptr : &upd);
    if (first && capture) KT(c, "capture", capture_pair<T>(c, pb, pz, qb, qz, s1, s2));
    KT(c, "fin_alpha", fin_alpha(c->partK, nbk, c->scal, c->flags, c->s));
    KT(c, PN(T, "cg_update"), cg_update<T>(xb, xz, pb, pz, qb, qz, rb, rz, zb, zz, s1, s2, pcc, c->scal, c->flags,
                                          n, c->partV, first, c->s));
    first = false;
    KT(c, "fin_rz", fin_rz(c->partV, nbv, c->scal, c->flags, c->s));
  }
}

// The chunk as a replayable HIP graph (recorded on first use; null when the
// runtime refuses, and the caller then queues the chunk directly).  The
// kernels and their arguments are the same as those pcg_chunk queues, so a
// replay computes exactly what the direct launches compute.
template <typename T>
hipGraphExec_t pcg_graph(csipm_ctx* c, int chunk, bool first, T* xb, T* xz, const T* s1, const T* s2,
                         const float* pcc) {
  // (a key whose recording failed is kept with a null exec: not retried)
  for (const auto& gr : c->graphs)
    if (gr.wbytes == (int)sizeof(T) && gr.chunk == chunk && gr.first == first && gr.pcc == pcc) return gr.exec;
  if (!c->cap_s && hipStreamCreateWithFlags(&c->cap_s, hipStreamNonBlocking) != hipSuccess) {
    c->cap_s = nullptr;
    return nullptr;
  }
  hipStream_t s0 = c->s;
  c->s = c->cap_s;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ok = hipStreamBeginCapture(c->cap_s, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    pcg_chunk<T>(c, chunk, first, xb, xz, s1, s2, pcc, false);
    ok = hipStreamEndCapture(c->cap_s, &graph) == hipSuccess && graph;
  }
  c->s = s0;
  if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
  if (graph) (void)hipGraphDestroy(graph);
  if (!ok) {
    const hipError_t e = hipGetLastError();
    c->err = std::string("pcg: graph recording failed, chunks are launched directly: ") + hipGetErrorString(e);
    exec = nullptr;
  }
  c->graphs.push_back({(int)sizeof(T), chunk, first, pcc, exec});
  return exec;
}

// PCG: chunks of 2, 4, 8 and 16 iterations between host reads of the
// stopping flag; with graphs (no timing, no capture) each chunk is one graph
// launch.
template <typename T>
csipm_status pcg(csipm_ctx* c, T* xb, T* xz, const T* s1, const T* s2, const float* pcc, PcgOut& out,
                 bool capture, bool graphs) {
  // the first chunk covers as many iterations as the last solve needed (a
  // power of two in [2, 16]), so that most systems need one host read;
  // queued iterations past convergence return at once
  int chunk = 2;
  while (chunk < c->pcg_hint && chunk < 16) chunk *= 2;
  bool first = true;
  // (a context's first solve launches directly: recording and first
  // replays cost more than one solve of a small grid gains)
  const bool use_graphs = graphs && !capture && !c->kt_on && c->solves > 0;
  for (;;) {
    hipGraphExec_t ex = use_graphs ? pcg_graph<T>(c, chunk, first, xb, xz, s1, s2, pcc) : nullptr;
    if (ex) {
      if (hipGraphLaunch(ex, c->s) != hipSuccess) return fail(c, CSIPM_EHIP, "pcg: graph launch failed");
    } else {
      pcg_chunk<T>(c, chunk, first, xb, xz, s1, s2, pcc, capture);
    }
    first = false;
    csipm_status st = sync_scalars(c, "pcg");
    if (st != CSIPM_OK) return st;
    if (c->hflags[F_DONE]) break;
    chunk = std::min(chunk * 2, 16);
  }
  out.iters = c->hflags[F_IT];
  out.breakdown = c->hflags[F_BREAK] != 0;
  out.res0 = std::sqrt(std::max(c->hscal[S_RZ0], 0.0));
  out.res = c->hscal[S_RES];
  out.converged = out.res <= c->hscal[S_TOL];
  c->pcg_hint = out.iters;
  return CSIPM_OK;
}

// Preconditioned conjugate residuals on K x = h from the same start as pcg
// (r = h and z = P^{-1}r in the Krylov vectors, finalised by
// k_fin_cg_init); stops on the same sqrt(r.P^{-1}r) test.  Per iteration:
// w = K z (with z.w), then p = z + beta p and q = w + beta q (with
// q.P^{-1}q), then the update of x, r and z = P^{-1}r that CG uses.
template <typename T>
csipm_status pcr(csipm_ctx* c, T* xb, T* xz, const T* s1, const T* s2, const float* pcc, PcgOut& out) {
  const long long n = c->g.n;
  PcgSet v = pcg_set<T>(c);
  T *rb = (T*)v.rb, *rz = (T*)v.rz, *zb = (T*)v.zb, *zz = (T*)v.zz, *pb = (T*)v.pb, *pz = (T*)v.pz,
    *qb = (T*)v.qb, *qz = (T*)v.qz, *work = (T*)v.work, *wb = (T*)v.wb, *wz = (T*)v.wz;
  const int nbv = vec_blocks(n);
  const int* skip = c->flags + F_DONE;
  int chunk = 2;
  bool first = true;
  for (;;) {
    for (int k = 0; k < chunk; ++k) {
      const int nbk = op_K<T>(c, zb, zz, s1, s2, wb, wz, work, skip);
      KT(c, "fin_cr_zw", fin_cr_zw(c->partK, nbk, c->scal, c->flags, first, c->s));
      KT(c, PN(T, "cr_dir"),
         cr_dir<T>(pb, pz, qb, qz, zb, zz, wb, wz, s1, s2, pcc, c->scal, c->flags, n, c->partV, first, c->s));
      KT(c, "fin_alpha", fin_alpha(c->partV, nbv, c->scal, c->flags, c->s));
      KT(c, PN(T, "cg_update"), cg_update<T>(xb, xz, pb, pz, qb, qz, rb, rz, zb, zz, s1, s2, pcc, c->scal, c->flags,
                                            n, c->partV, first, c->s));
      first = false;
      KT(c, "fin_rz", fin_rz(c->partV, nbv, c->scal, c->flags, c->s));
    }
    csipm_status st = sync_scalars(c, "pcr");
    if (st != CSIPM_OK) return st;
    if (c->hflags[F_DONE]) break;
    chunk = std::min(chunk * 2, 16);
  }
  out.iters = c->hflags[F_IT];
  out.breakdown = c->hflags[F_BREAK] != 0;
  out.res0 = std::sqrt(std::max(c->hscal[S_RZ0], 0.0));
  out.res = c->hscal[S_RES];
  out.converged = out.res <= c->hscal[S_TOL];
  return CSIPM_OK;
}

// Preconditioned conjugate A-residuals on K x = h, x0 = 0: the caller has
// put z = P^{-1}h into the Krylov set (and r = h, which CAr overwrites with
// u).  Start: w = K z, u = P^{-1} w.  Each iteration: s = K u (partial u.s),
// beta and alpha's numerator u.s (fin_cr_zw), the direction step
// (car_dir: p, v = P^{-1}Kp, y = P^{-1}Kv; partial y.Py = t.P^{-1}t),
// alpha, the update (car_update: x, z, u; partial z.Pz = r.P^{-1}r) and the
// stopping test on sqrt(r.P^{-1}r) (fin_rz).  Vectors: u in r's place
// (r = P z is written back at the end), v in q's, s in w's, y in its own.
template <typename T>
csipm_status pcar(csipm_ctx* c, T* xb, T* xz, const T* s1, const T* s2, const float* pcc, PcgOut& out) {
  const long long n = c->g.n;
  PcgSet v = pcg_set<T>(c);
  T *ub = (T*)v.rb, *uz = (T*)v.rz, *zb = (T*)v.zb, *zz = (T*)v.zz, *pb = (T*)v.pb, *pz = (T*)v.pz,
    *vb = (T*)v.qb, *vz = (T*)v.qz, *work = (T*)v.work, *sb = (T*)v.wb, *sz = (T*)v.wz, *yb = (T*)v.yb,
    *yz = (T*)v.yz;
  const int nbv = vec_blocks(n);
  const int* skip = c->flags + F_DONE;
  // w = K z into s's buffer, then u = P^{-1} w (skipped when the solve is
  // already done at initialisation: the first update then writes x = 0)
  (void)op_K<T>(c, zb, zz, s1, s2, sb, sz, work, skip);
  KT(c, PN(T, "pinv"), pinv_apply<T>(sb, sz, ub, uz, s1, s2, pcc, n, c->partV, nullptr, c->s));
  int chunk = 2;
  bool first = true;
  for (;;) {
    for (int k = 0; k < chunk; ++k) {
      const int nbk = op_K<T>(c, ub, uz, s1, s2, sb, sz, work, skip);
      KT(c, "fin_cr_zw", fin_cr_zw(c->partK, nbk, c->scal, c->flags, first, c->s));
      KT(c, PN(T, "car_dir"), car_dir<T>(pb, pz, vb, vz, yb, yz, zb, zz, ub, uz, sb, sz, s1, s2, pcc, c->scal,
                                         c->flags, n, c->partV, first, c->s));
      KT(c, "fin_alpha", fin_alpha(c->partV, nbv, c->scal, c->flags, c->s));
      KT(c, PN(T, "car_update"), car_update<T>(xb, xz, pb, pz, zb, zz, vb, vz, ub, uz, yb, yz, s1, s2, pcc,
                                               c->scal, c->flags, n, c->partV, first, c->s));
      first = false;
      KT(c, "fin_rz", fin_rz(c->partV, nbv, c->scal, c->flags, c->s));
    }
    csipm_status st = sync_scalars(c, "pcar");
    if (st != CSIPM_OK) return st;
    if (c->hflags[F_DONE]) break;
    chunk = std::min(chunk * 2, 16);
  }
  // the residual r = P z back into r's place (u is no longer needed): the
  // interior-point update recovers H d_beta from it
  KT(c, PN(T, "p_apply"), p_apply<T>(zb, zz, s1, s2, pcc, ub, uz, n, c->s));
  out.iters = c->hflags[F_IT];
  out.breakdown = c->hflags[F_BREAK] != 0;
  out.res0 = std::sqrt(std::max(c->hscal[S_RZ0], 0.0));
  out.res = c->hscal[S_RES];
  out.converged = out.res <= c->hscal[S_TOL];
  return CSIPM_OK;
}

// The Newton systems' Krylov method (options.krylov); capture needs CG.
template <typename T>
csipm_status krylov(csipm_ctx* c, int method, T* xb, T* xz, const T* s1, const T* s2, const float* pcc, PcgOut& out,
                    bool capture, bool graphs) {
  if (method == CSIPM_KRYLOV_CR) return pcr<T>(c, xb, xz, s1, s2, pcc, out);
  if (method == CSIPM_KRYLOV_CAR) return pcar<T>(c, xb, xz, s1, s2, pcc, out);
  return pcg<T>(c, xb, xz, s1, s2, pcc, out, capture, graphs);
}

}  // namespace

// ---------------------------------------------------------------- C-ABI --
extern "C" {

void csipm_default_options(csipm_options* o) {
  if (!o) return;
  o->tol = 1e-6;
  o->max_iter = 200;
  o->cg_max = 500;
  o->cg_rtol = 1e-2;
  o->cg_atol = 0.0;
  o->sigma = 0.1;
  o->tau = 0.99;
  o->precision = CSIPM_FP64;
  o->pc = CSIPM_PC_PLAIN;
  o->refine_max = 8;
  o->refine_inner_rtol = 1e-5;
  o->refine_trust = 2e-6;
  o->pc_min_cg = 2;
  o->krylov = CSIPM_KRYLOV_CG;
  o->pc_rho = 0.0;
  o->pc_max_relevant = 0.5;
  o->mehrotra = 0;
  o->build_next = 1;
  o->graphs = 1;
  o->pc_min_missing = 0.01;
}

size_t csipm_workspace_bytes(int n1, int n2, int n3) {
  if (!fft_extent_supported(n1, 1) || !fft_extent_supported(n2, 2) || !fft_extent_supported(n3, 3)) return 0;
  csipm_ctx tmp;
  Carver cv{nullptr, 0, 0};
  return layout(cv, &tmp, n1, n2, n3);
}

csipm_status csipm_create(csipm_ctx** out, int n1, int n2, int n3, const double* d_signal,
                          const uint8_t* d_observed, void* d_workspace, size_t workspace_bytes, void* hip_stream) {
  if (!out) return CSIPM_EINVAL;
  *out = nullptr;
  if (!d_signal || !d_observed || !d_workspace) return CSIPM_EINVAL;
  if (!fft_extent_supported(n1, 1) || !fft_extent_supported(n2, 2) || !fft_extent_supported(n3, 3)) return CSIPM_EUNSUPPORTED;
  if ((reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0) return CSIPM_EINVAL;
  const size_t need = csipm_workspace_bytes(n1, n2, n3);
  if (workspace_bytes < need) return CSIPM_ENOMEM;
  const auto t_create = std::chrono::steady_clock::now();
  csipm_ctx* c = new (std::nothrow) csipm_ctx();
  if (!c) return CSIPM_ENOMEM;
  c->g = make_grid(n1, n2, n3);
  c->s = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return CSIPM_EHIP;
  }
  Carver cv{reinterpret_cast<char*>(d_workspace), 0, workspace_bytes};
  layout(cv, c, n1, n2, n3);
  if (hipHostMalloc((void**)&c->hscal, sizeof(double) * S_COUNT + sizeof(int) * F_COUNT) != hipSuccess) {
    delete c;
    return CSIPM_EHIP;
  }
  c->hflags = reinterpret_cast<int*>(c->hscal + S_COUNT);
  const Grid& g = c->g;
  const long long n = g.n;

  // twiddle tables exp(-2 pi i q / L), from long double, rounded once
  const int Ls[4] = {n1, n2, n3 / 2, n3};
  std::vector<cx<double>> h64;
  std::vector<cx<float>> h32;
  for (int L : Ls)
    for (int q = 0; q < L; ++q) {
      const long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)q / (long double)L;
      const long double cr = cosl(a), ci = sinl(a);
      h64.push_back({(double)cr, (double)ci});
      h32.push_back({(float)cr, (float)ci});
    }
  hipError_t e = hipMemcpyAsync(c->tw64, h64.data(), h64.size() * sizeof(cx<double>), hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->tw32, h32.data(), h32.size() * sizeof(cx<float>), hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess) e = hipStreamSynchronize(c->s);
  if (e != hipSuccess) {
    noctx_set_error(std::string("create: twiddle tables: ") + hipGetErrorString(e));
    (void)hipHostFree(c->hscal);
    delete c;
    return CSIPM_EHIP;
  }
  size_t o = 0;
  c->T64.t1 = c->tw64 + o; c->T32.t1 = c->tw32 + o; o += n1;
  c->T64.t2 = c->tw64 + o; c->T32.t2 = c->tw32 + o; o += n2;
  c->T64.tm = c->tw64 + o; c->T32.tm = c->tw32 + o; o += n3 / 2;
  c->T64.t3 = c->tw64 + o; c->T32.t3 = c->tw32 + o;

  // input checks: finite observed samples, at least one observed
  const long long nr = g.nr;   // real-space samples (n beta coordinates)
  check_signal(d_signal, d_observed, nr, c->partV, c->scal + S_SIG, c->s);
  csipm_status st = sync_scalars(c, "create");
  if (st != CSIPM_OK) { noctx_set_error("create: " + c->err); csipm_destroy(c); return st; }
  if (c->hscal[S_SIG] > 0) { csipm_destroy(c); return CSIPM_ENONFINITE; }
  c->nobs = (long long)c->hscal[S_SIG + 1];
  if (c->nobs == 0) { csipm_destroy(c); return CSIPM_EINVAL; }

  launch_pack_mask(g, d_observed, c->mask, c->s);
  // xi = A^T b_hat (b_hat: zero-filled signal, staged in rb as a real grid)
  zero_fill(d_signal, d_observed, c->rb, nr, c->s);
  op_At<double>(c, c->rb, c->xi, c->work);
  absmax(c->xi, n, c->partV, c->scal + S_MISC, c->s);
  // diag(M_perp^T M_perp) from A^T(mask), through the external layout (the
  // coordinate without data, if any, gets 0)
  obs_to_double(d_observed, c->rb, nr, c->s);
  op_At<double>(c, c->rb, c->zb, c->work);
  launch_to_external<double, double>(g, c->zb, c->zz, c->s);
  diag_h(c->zz, c->rz, n1, n2, n3, (double)c->nobs / (double)nr, c->s);
  launch_to_internal<double, double>(g, c->rz, c->diagH, c->s);
  fill<float>(c->pc_c, 1.0f, n, c->s);
  st = sync_scalars(c, "create");
  if (st != CSIPM_OK) { noctx_set_error("create: " + c->err); csipm_destroy(c); return st; }
  c->xi_inf = c->hscal[S_MISC];
  // barrier diagonals default to 1 so apply_K / apply_Pinv are defined
  fill<double>(c->sig1, 1.0, n, c->s);
  fill<double>(c->sig2, 1.0, n, c->s);
  fill<float>(c->sig1f, 1.0f, n, c->s);
  fill<float>(c->sig2f, 1.0f, n, c->s);
  st = sync_scalars(c, "create");
  if (st != CSIPM_OK) { noctx_set_error("create: " + c->err); csipm_destroy(c); return st; }
  c->setup_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_create).count();
  *out = c;
  return CSIPM_OK;
}

csipm_status csipm_set_lambda(csipm_ctx* c, double lambda) {
  if (!c) return CSIPM_EINVAL;
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(c, CSIPM_EINVAL, "lambda must be finite and > 0");
  c->lambda = lambda;
  c->have_lambda = true;
  return CSIPM_OK;
}

csipm_status csipm_lambda_rule(csipm_ctx* c, double frac, double* lambda_out) {
  if (!c) return CSIPM_EINVAL;
  if (!(frac > 0.0) || !std::isfinite(frac)) return fail(c, CSIPM_EINVAL, "frac must be finite and > 0");
  if (!(c->xi_inf > 0.0)) return fail(c, CSIPM_EINVAL, "M_perp^T b is zero: every lambda > 0 gives beta = 0");
  c->lambda = frac * c->xi_inf;
  c->have_lambda = true;
  if (lambda_out) *lambda_out = c->lambda;
  return CSIPM_OK;
}

namespace {

// Builds and solves the Newton system of the current iterate (target
// smu = sigma mu): K [dxb; dxz] = h with the barrier diagonals Sigma_j =
// nu_j / s_j, either by FP64 PCG or by FP32 PCG inside FP64 iterative
// refinement.  The system build is fused with the PCG start (newton_init).
// Where the iterate update finds H d_beta after a Newton solve.
enum HdSource {
  HD_RRES64,   // recovered from the FP64 PCG residual (rb, rz)
  HD_DIRECT,   // written by the FP64 refinement residual pass (rb)
  HD_RRES32    // recovered from the FP32 PCG residual (frb, frz): FP32-level accuracy
};

csipm_status newton_solve(csipm_ctx* c, const csipm_options& o, double smu, double eta, const float* pcc,
                          int& cg_iters, int& refine_steps, bool& converged, bool capture, HdSource& src,
                          const double* dab = nullptr, const double* daz = nullptr, bool prebuilt = false) {
  const long long n = c->g.n;
  const int nbv = vec_blocks(n);
  // a system built by the previous iterate update (prebuilt) left its r.z
  // and h.P^{-1}h partials after the residual quantities
  double* const part0 = prebuilt ? c->partV + (size_t)NRESID_Q * VEC_MAX_BLOCKS : c->partV;
  cg_iters = 0;
  refine_steps = 0;
  converged = false;
  src = HD_RRES64;
  // CG starts from p = z and overwrites z before reading it
  const bool cg = o.krylov == CSIPM_KRYLOV_CG;
  if (o.precision == CSIPM_FP64) {
    if (!prebuilt)
      KT(c, "newton_init.f64",
         newton_init<double>(c->beta, c->z, c->nu1, c->nu2, c->hb, c->lambda, smu, c->sig1, c->sig2, nullptr,
                             nullptr, nullptr, nullptr, pcc, c->rb, c->rz, cg ? nullptr : c->zb, c->zz, c->pb, c->pz,
                             n, c->partV, c->s, dab, daz));
    KT(c, "fin_cg_start",
       fin_cg_start(part0, nbv, VEC_MAX_BLOCKS, c->scal, c->flags, eta, o.cg_atol, o.cg_max, -1, -1, c->s));
    PcgOut po;
    csipm_status st = krylov<double>(c, o.krylov, c->dxb, c->dxz, c->sig1, c->sig2, pcc, po, capture, o.graphs != 0);
    cg_iters = po.iters;
    converged = po.converged;
    return st;
  }
  // FP32 inner solves, FP64 residual: d = 0, r = h; repeat { e = K32^{-1} r;
  // d += e; r = h - K d } until sqrt(r.P^{-1}r) <= max(atol, eta sqrt(h.P^{-1}h)).
  // The first inner solve starts from h (built in FP32 by newton_init, which
  // also sums h.P^{-1}h); later ones start from the FP32 residual (built
  // from the fused FP64 residual pass by ref_restart).  A system whose
  // tolerance is loose enough for FP32 (eta >= refine_trust) takes the FP32
  // solution to half its tolerance without the FP64 residual pass.
  const bool trusted = o.refine_trust > 0.0 && eta >= o.refine_trust;
  // (an unrefined system stores no FP64 Sigma or h: nothing reads them,
  // except the features of a capture)
  if (!prebuilt)
    KT(c, trusted ? "newton_init_noh.f32" : "newton_init.f32",
       newton_init<float>(c->beta, c->z, c->nu1, c->nu2, c->hb, c->lambda, smu,
                          trusted && !capture ? nullptr : c->sig1, trusted && !capture ? nullptr : c->sig2,
                          trusted ? nullptr : c->rhb, trusted ? nullptr : c->rhz, c->sig1f, c->sig2f, pcc, c->frb,
                          c->frz, cg ? nullptr : c->fzb, c->fzz, c->fpb, c->fpz, n, c->partV, c->s, dab, daz));
  // inner tolerance: half the remaining reduction, at most 1e-2, at least
  // refine_inner_rtol (what FP32 PCG can still reach)
  double inner = std::max(o.refine_inner_rtol, std::min(1e-2, 0.5 * eta));
  if (trusted) {
    KT(c, "fin_cg_start",
       fin_cg_start(part0, nbv, VEC_MAX_BLOCKS, c->scal, c->flags, inner, 0.0, o.cg_max, -1, -1, c->s));
    PcgOut po;
    csipm_status st = krylov<float>(c, o.krylov, c->fxb, c->fxz, c->sig1f, c->sig2f, pcc, po, capture, o.graphs != 0);
    if (st != CSIPM_OK) return st;
    cg_iters = po.iters;
    converged = po.converged;
    src = HD_RRES32;   // the step is read from the FP32 solution itself
    return CSIPM_OK;
  }
  src = HD_DIRECT;
  KT(c, "fin_cg_start",
     fin_cg_start(part0, nbv, VEC_MAX_BLOCKS, c->scal, c->flags, inner, 0.0, o.cg_max, S_REF0, -1, c->s));
  double target = 0.0, rnorm = 0.0;
  double prev_rnorm = INFINITY, prev_rinf = INFINITY;
  int first_iters = 0;
  for (int step = 0; step < std::max(1, o.refine_max); ++step) {
    // a later inner solve gets at most max(50, 2x the first one's) iterations:
    // one that needs more is stuck at FP32 resolution of a tiny residual
    const int inner_max = step == 0 ? o.cg_max : std::min(o.cg_max, std::max(50, 2 * first_iters));
    if (step > 0)
      KT(c, "fin_cg_start",
         fin_cg_start(nullptr, 0, 0, c->scal, c->flags, inner, 0.0, inner_max, -1, S_REFRZ, c->s));
    PcgOut po;
    csipm_status st =
        krylov<float>(c, o.krylov, c->fxb, c->fxz, c->sig1f, c->sig2f, pcc, po, capture && step == 0, o.graphs != 0);
    if (st != CSIPM_OK) return st;
    cg_iters += po.iters;
    if (step == 0)
      KT(c, "set_f2d", set_f2d(c->dxb, c->dxz, c->fxb, c->fxz, n, c->s));
    else
      KT(c, "add_f2d", add_f2d(c->dxb, c->dxz, c->fxb, c->fxz, n, c->s));
    op_Kr(c, pcc);
    st = sync_scalars(c, "refine");
    if (st != CSIPM_OK) return st;
    ++refine_steps;
    const double h0 = std::sqrt(std::max(c->hscal[S_REF0], 0.0));
    target = std::max(o.cg_atol, eta * h0);
    rnorm = std::sqrt(std::max(c->hscal[S_REF], 0.0));
    // besides the preconditioned norm, every component of r must be below
    // eta in the KKT residual's scale: an FP32 solution misrepresents
    // d_beta + d_z where one slack is tiny and its Sigma huge, which leaves
    // single large components that a global norm over n values can hide
    const double rinf = c->hscal[S_REFINF];
    if (rnorm <= target && rinf <= eta * (1.0 + c->xi_inf)) {
      converged = true;
      break;
    }
    if (step == 0) first_iters = po.iters;
    // stop at the precision floor: a step that halves neither measure of r
    // will not be followed by one that does
    const bool progress = rnorm < 0.5 * prev_rnorm || rinf < 0.5 * prev_rinf;
    prev_rnorm = rnorm;
    prev_rinf = rinf;
    if (po.iters == 0 || !std::isfinite(rnorm) || !progress || step + 1 >= std::max(1, o.refine_max)) break;
    const double need = std::min(target / rnorm, rinf > 0.0 ? eta * (1.0 + c->xi_inf) / rinf : 1.0);
    inner = std::max(o.refine_inner_rtol, std::min(1e-2, 0.5 * need));
    // FP32 start of the next inner solve: r32, z32 = p32 = P_c^{-1} r, r32.z32 -> S_REFRZ
    KT(c, "ref_restart+fin",
       ref_restart(c->rhb, c->rhz, c->dxb, c->dxz, c->rb, c->sig1, c->sig2, pcc, c->frb, c->frz,
                   cg ? nullptr : c->fzb, c->fzz, c->fpb, c->fpz, n, c->partV, c->scal + S_REFRZ, c->s));
  }
  return CSIPM_OK;
}

// two FP64 n-arrays copied on the context's stream
void copy_pair(double* db, double* dz, const double* sb, const double* sz, long long n, hipStream_t s) {
  const size_t b = sizeof(double) * (size_t)n;
  (void)hipMemcpyAsync(db, sb, b, hipMemcpyDeviceToDevice, s);
  (void)hipMemcpyAsync(dz, sz, b, hipMemcpyDeviceToDevice, s);
}

// (beta, z, nu1, nu2) <-> snap
void save_state(csipm_ctx* c) {
  const size_t b = sizeof(double) * (size_t)c->g.n;
  const double* src[4] = {c->beta, c->z, c->nu1, c->nu2};
  for (int i = 0; i < 4; ++i) (void)hipMemcpyAsync(c->snap + i * c->g.n, src[i], b, hipMemcpyDeviceToDevice, c->s);
}
void restore_state(csipm_ctx* c) {
  const size_t b = sizeof(double) * (size_t)c->g.n;
  double* dst[4] = {c->beta, c->z, c->nu1, c->nu2};
  for (int i = 0; i < 4; ++i) (void)hipMemcpyAsync(dst[i], c->snap + i * c->g.n, b, hipMemcpyDeviceToDevice, c->s);
}

struct Resid {
  double fb, fz, cmax, csum, bmax, pmin, nonfinite;
  double relevant;   // coefficients where the learned correction can matter (when reduced)
  double dscale;     // after a carried update from rres: max (S1 + S2)(|d_beta| + |d_z|)
};

// Residual parts last reduced into scal[S_RESID..] (after a sync).
Resid read_resid(const csipm_ctx* c) {
  const double* v = c->hscal + S_RESID;
  return Resid{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[8], v[9]};
}

// Residual parts with G = H beta - xi recomputed by a full H-apply (and the
// sum of log(S1 + S2) into scal[S_RESID + 7] when logsum).
csipm_status residuals(csipm_ctx* c, Resid& r, bool logsum) {
  op_H<double>(c, c->beta, c->hb, c->work);
  KT(c, "ipm_resid+fin", ipm_resid(c->beta, c->z, c->nu1, c->nu2, c->hb, c->xi, c->lambda, c->g.n, c->partV,
                                    c->scal + S_RESID, logsum, c->s));
  csipm_status st = sync_scalars(c, "residuals");
  if (st != CSIPM_OK) return st;
  r = read_resid(c);
  return CSIPM_OK;
}

// The learned correction of the current iterate when the last iterate update
// has built its Newton system with the paper's P (in FP64, or in FP32 with
// or without the FP64 h and Sigma of a refined solve): c from the state (as learned_correction forms
// it), and the PCG start and its sums rewritten to those of P_c, so that no
// newton_init pass rebuilds the system.  The update's residual reduction has
// left the centring sum and max |beta| of this iterate, and its activity
// flags the chunks where the correction's gate passes: only those chunks,
// and those where c was last set, are visited.
csipm_status correction_patch(csipm_ctx* c, bool f64, bool ref64) {
  const long long n = c->g.n;
  const int nbv = vec_blocks(n);
  double* const part = c->partV + (size_t)NRESID_Q * VEC_MAX_BLOCKS;
  const double* ml = c->scal + S_RESID + 7;
  const double* bmax = c->scal + S_RESID + 4;
  const double mscale = 1.0 / (double)n;
  if (f64) {
    KT(c, "correction_patch.f64",
       mlp_correction_patch<double>(c->beta, c->z, c->nu1, c->nu2, c->diagH, ml, mscale, bmax, c->mlp_params, c->pc_c,
                                    n, c->pc_act, c->pc_set, c->pc_tracked, c->sig1, c->sig2, c->rb, c->rz, c->pb,
                                    c->pz, nullptr, nullptr, nullptr, nullptr, part, VEC_MAX_BLOCKS, nbv, c->s));
  } else {
    KT(c, "correction_patch.f32",
       mlp_correction_patch<float>(c->beta, c->z, c->nu1, c->nu2, c->diagH, ml, mscale, bmax, c->mlp_params, c->pc_c,
                                   n, c->pc_act, c->pc_set, c->pc_tracked, c->sig1f, c->sig2f, c->frb, c->frz, c->fpb,
                                   c->fpz, ref64 ? c->sig1 : nullptr, ref64 ? c->sig2 : nullptr,
                                   ref64 ? c->rhb : nullptr, ref64 ? c->rhz : nullptr, part, VEC_MAX_BLOCKS, nbv,
                                   c->s));
  }
  c->pc_tracked = true;
  return hip_check(c, "correction_patch");
}

// LASSO certificate of beta from G = H beta - xi (which must be exact: an
// FP64 H-apply, not the carried value) into the certificate fields of inf;
// synchronises.
csipm_status certificate(csipm_ctx* c, csipm_info& inf) {
  KT(c, "lasso_cert+fin", lasso_cert(c->beta, c->hb, c->lambda, c->g.n, c->partV, c->scal + S_CERT, c->s));
  csipm_status st = sync_scalars(c, "certificate");
  if (st != CSIPM_OK) return st;
  const double* q = c->hscal + S_CERT;
  const double rr = q[0], l1 = q[1], termwise = q[2], bG = q[3], ginf = q[4], nat = q[5], bmax = q[6];
  const double lam = c->lambda;
  // dual point theta = s r, scaled into ||M_perp^T theta||_inf <= lambda
  const double sc = ginf > lam ? lam / ginf : 1.0;
  const double bg = -bG;   // beta.g with g = -G
  inf.objective = 0.5 * rr + lam * l1;
  inf.dual_objective = sc * (rr + bg) - 0.5 * sc * sc * rr;
  const double gap = 0.5 * (1.0 - sc) * (1.0 - sc) * rr + termwise + (1.0 - sc) * bg;
  inf.rel_dual_gap = gap / std::max(std::fabs(inf.objective), 1e-300);
  inf.natural_residual = nat / std::max(1.0, bmax);
  inf.g_inf = ginf;
  inf.setup_seconds = c->setup_s;
  return CSIPM_OK;
}

// G = H beta - xi is carried from iteration to iteration (k_ipm_advance: G +=
// alpha H d_beta); it is
// recomputed by a full H-apply before a stopping decision, at least every
// kExactEvery iterations, and before the first FP32 Newton system that is
// refined after unrefined ones, so carried error never accumulates far.
constexpr int kExactEvery = 16;
// H beta recovered from an FP64 Krylov residual (h - r minus the Sigma terms
// of d) carries rounding of order eps (S1 + S2)(|d_beta| + |d_z|), which
// grows as the slacks close; H beta is also recomputed once the accumulated
// bound exceeds this fraction of the KKT residual, so that the Newton
// right-hand side stays accurate far inside the Krylov tolerance
constexpr double kCarryFrac = 0.01;
// the solve stops (CSIPM_STALLED) once rel_kkt exceeds this multiple of the
// best value it reached
constexpr double kStallFactor = 10.0;

}  // namespace

csipm_status csipm_solve(csipm_ctx* c, const csipm_options* opts, csipm_info* info) {
  if (!c) return CSIPM_EINVAL;
  if (!c->have_lambda) return fail(c, CSIPM_ESTATE, "lambda not set");
  csipm_options o;
  csipm_default_options(&o);
  if (opts) o = *opts;
  if (!(o.tol > 0) || o.max_iter < 0 || o.cg_max < 1 || !(o.sigma > 0 && o.sigma < 1) || !(o.tau > 0 && o.tau < 1) ||
      (o.precision != CSIPM_FP64 && o.precision != CSIPM_FP32) ||
      (o.pc != CSIPM_PC_PLAIN && o.pc != CSIPM_PC_LEARNED && o.pc != CSIPM_PC_SCALED) ||
      (o.krylov != CSIPM_KRYLOV_CG && o.krylov != CSIPM_KRYLOV_CR && o.krylov != CSIPM_KRYLOV_CAR) || !(o.pc_rho >= 0.0) ||
      !(o.pc_max_relevant >= 0.0 && o.pc_max_relevant <= 1.0) || (o.mehrotra != 0 && o.mehrotra != 1) ||
      (o.build_next != 0 && o.build_next != 1) || (o.graphs != 0 && o.graphs != 1) ||
      !(o.refine_trust >= 0.0 && o.refine_trust <= 1.0) || !(o.refine_inner_rtol > 0.0) || o.pc_min_cg < 0 ||
      !(o.pc_min_missing >= 0.0 && o.pc_min_missing <= 1.0))
    return fail(c, CSIPM_EINVAL, "invalid options");
  if (o.pc == CSIPM_PC_LEARNED && !c->have_params) return fail(c, CSIPM_ESTATE, "learned preconditioner has no parameters");
  const auto t0 = std::chrono::steady_clock::now();
  const long long n = c->g.n;
  const double lam = c->lambda;
  c->log.clear();
  c->cap_count = 0;
  c->cap_cg.clear();
  const double z0 = c->xi_inf > 0 ? c->xi_inf : 1.0;
  // the learned form acts only within the missing fractions its network
  // was trained on; below pc_min_missing it is the paper's P throughout
  const double missing = 1.0 - (double)c->nobs / (double)c->g.nr;
  const bool in_domain = missing >= o.pc_min_missing;
  const bool learned = o.pc == CSIPM_PC_LEARNED && in_domain;
  // the residual passes count the coefficients where the correction can act
  // (and sum the centring of its first feature) for the learned form and for
  // a capture that follows the correction's policy
  const bool need_rel = learned || (c->cap_enable == 2 && in_domain);
  // scaled identity: c = rho everywhere, rho = m/n unless given
  const float* pc_fixed = nullptr;
  if (o.pc == CSIPM_PC_SCALED) {
    const double rho = o.pc_rho > 0.0 ? o.pc_rho : (double)c->nobs / (double)n;
    KT(c, "fill", fill<float>(c->pc_c, (float)rho, n, c->s));
    c->pc_tracked = false;
    pc_fixed = c->pc_c;
  }
  // the start beta = 0 has H beta = 0 exactly: G = -xi
  KT(c, "ipm_init", ipm_init(c->beta, c->z, c->nu1, c->nu2, c->hb, c->xi, n, z0, lam, c->s));
  KT(c, "ipm_resid+fin",
     ipm_resid(c->beta, c->z, c->nu1, c->nu2, c->hb, nullptr, lam, n, c->partV, c->scal + S_RESID, need_rel, c->s));
  csipm_status st = sync_scalars(c, "solve start");
  if (st != CSIPM_OK) return st;
  Resid r = read_resid(c);
  bool exact = true;
  bool approx = false;   // carried H beta holds FP32-level error (an unrefined FP32 step)
  int carried = 0;
  double carry_err = 0.0;   // bound on the error of the carried H beta (max norm)
  double best_rel = INFINITY;
  bool have_snap = false;
  double snap_rel = INFINITY;
  // FP32 steps taken without refinement (refine_trust) are revoked for the
  // rest of the solve the first time the solve would stall after one: the
  // step is undone (or the solve goes on from the current iterate) and every
  // later Newton system is refined
  int unrefined_steps = 0;
  bool trust_revoked = false;
  auto revoke_trust = [&]() {
    if (trust_revoked || unrefined_steps == 0 || !(o.refine_trust > 0.0)) return false;
    o.refine_trust = 0.0;
    trust_revoked = true;
    return true;
  };
  csipm_info inf{};
  inf.lambda = lam;
  inf.xi_inf = c->xi_inf;
  csipm_status result = CSIPM_NOT_CONVERGED;
  int prev_cg = 0;
  // the Newton system the last iterate update built for the next iteration
  // (see the step below): none, FP32 without / with the FP64 refinement
  // arrays, or FP64
  enum { NEXT_NONE = 0, NEXT_F32 = 1, NEXT_F32_REF = 2, NEXT_F64 = 3 };
  int next_kind = NEXT_NONE;
  double prev_rel = INFINITY;
  for (int it = 0;; ++it) {
    auto rel_of = [&](const Resid& q) { return std::max(std::max(q.fb, q.fz), q.cmax) / (1.0 + c->xi_inf); };
    double rel = rel_of(r);
    const bool leaving_trust = approx && !(std::min(o.cg_rtol, 0.1 * rel) >= o.refine_trust);
    if (!exact && (rel <= o.tol || it >= o.max_iter || carried >= kExactEvery || leaving_trust || have_snap ||
                   carry_err > kCarryFrac * rel * (1.0 + c->xi_inf) || rel > kStallFactor * best_rel ||
                   !std::isfinite(rel))) {
      st = residuals(c, r, need_rel);
      if (st != CSIPM_OK) return st;
      exact = true;
      approx = false;
      carried = 0;
      carry_err = 0.0;
      rel = rel_of(r);
      next_kind = NEXT_NONE;   // built from the carried G
    }
    // a step along an inexact direction (the Newton solve stopped at its
    // precision floor or budget) that raised rel_kkt is undone, and the solve
    // ends there with the better iterate
    if (have_snap && !(rel <= snap_rel)) {
      restore_state(c);
      st = residuals(c, r, need_rel);
      if (st != CSIPM_OK) return st;
      rel = rel_of(r);
      exact = true;
      approx = false;
      carried = 0;
      carry_err = 0.0;
      next_kind = NEXT_NONE;   // (built from the undone iterate)
      if (!revoke_trust()) {
        result = CSIPM_STALLED;
        inf.rel_kkt = rel;
        inf.res_beta_inf = r.fb;
        inf.res_z_inf = r.fz;
        inf.compl_max = r.cmax;
        inf.mu = r.csum / (2.0 * (double)n);
        break;
      }
    }
    have_snap = false;
    if (r.nonfinite > 0 || !std::isfinite(r.fb)) return fail(c, CSIPM_ENONFINITE, "non-finite interior-point iterate");
    // past the precision floor the Newton steps stop reducing the residual
    // and start raising it: stop there rather than run into overflow
    if (rel > kStallFactor * best_rel && !revoke_trust()) {
      result = CSIPM_STALLED;
      inf.rel_kkt = rel;
      inf.res_beta_inf = r.fb;
      inf.res_z_inf = r.fz;
      inf.compl_max = r.cmax;
      inf.mu = r.csum / (2.0 * (double)n);
      if (!c->log.empty()) c->log.back().alpha = c->hscal[S_ALPHA_IPM];
      break;
    }
    best_rel = std::min(best_rel, rel);
    const double mu = r.csum / (2.0 * (double)n);
    inf.rel_kkt = rel;
    inf.res_beta_inf = r.fb;
    inf.res_z_inf = r.fz;
    inf.compl_max = r.cmax;
    inf.mu = mu;
    if (!c->log.empty()) c->log.back().alpha = c->hscal[S_ALPHA_IPM];
    if (rel <= o.tol) {
      result = inf.fallbacks > 0 ? CSIPM_FELL_BACK : CSIPM_OK;
      break;
    }
    if (it >= o.max_iter) {
      result = CSIPM_NOT_CONVERGED;
      break;
    }
    const double eta = std::min(o.cg_rtol, 0.1 * rel);
    int cgi = 0, ref = 0;
    bool conv = false, fell = false;
    HdSource src = HD_RRES64;
    // (a policy capture takes only the iterations where the learned form
    // would apply the correction: see use_learned below)
    const bool capture = c->cap_enable && o.pc == CSIPM_PC_PLAIN && o.krylov == CSIPM_KRYLOV_CG &&
                         c->cap_count < c->cap_max &&
                         (c->cap_enable != 2 || (in_domain && prev_cg >= o.pc_min_cg && r.relevant >= 1.0 &&
                                                 r.relevant / (double)n <= o.pc_max_relevant));
    // the correction is applied once a Newton system has needed more than
    // pc_min_cg - 1 PCG iterations (a system the paper's P solves in one
    // iteration leaves nothing to gain) and while at most pc_max_relevant of
    // the coefficients are relevant (reduced with the residual of the
    // iterate)
    const double relevant = need_rel ? r.relevant / (double)n : -1.0;
    const bool use_learned = learned && prev_cg >= o.pc_min_cg && relevant <= o.pc_max_relevant;
    // the system the last update built applies when it was built for this
    // precision and preconditioner
    const bool trusted_now = o.refine_trust > 0.0 && eta >= o.refine_trust;
    // (built with the paper's P: with the correction it is patched in place)
    const bool prebuilt = !o.mehrotra &&
                          (next_kind == NEXT_F64   ? o.precision == CSIPM_FP64
                           : next_kind == NEXT_F32_REF ? o.precision == CSIPM_FP32
                           : next_kind == NEXT_F32     ? o.precision == CSIPM_FP32 && trusted_now
                                                       : false);
    const int built_kind = next_kind;
    next_kind = NEXT_NONE;
    if (use_learned) {
      st = prebuilt ? correction_patch(c, built_kind == NEXT_F64, built_kind == NEXT_F32_REF)
                    : learned_correction(c, true);
      if (st != CSIPM_OK) return st;
    }
    // one Newton system at target tmu (with the corrector terms of the affine
    // direction when dab is set): the learned correction within a budget and
    // the paper's P as its fallback, or the plain / scaled P
    auto solve_system = [&](double tmu, const double* dab, const double* daz, bool cap) -> csipm_status {
      int a = 0, b = 0;
      csipm_status e;
      if (use_learned) {
        csipm_options ol = o;
        const int budget = prev_cg > 0 ? std::min(o.cg_max, std::max(8, (prev_cg * 3) / 2)) : o.cg_max;
        ol.cg_max = budget;
        e = newton_solve(c, ol, tmu, eta, c->pc_c, a, b, conv, false, src, dab, daz, prebuilt);
        if (e != CSIPM_OK) return e;
        cgi += a;
        ref += b;
        if (!conv) {   // (rebuilt with the paper's P)
          e = newton_solve(c, o, tmu, eta, nullptr, a, b, conv, false, src, dab, daz);
          if (e != CSIPM_OK) return e;
          cgi += a;
          ref += b;
          fell = true;
          ++inf.fallbacks;
        }
      } else {
        e = newton_solve(c, o, tmu, eta, pc_fixed, a, b, conv, cap, src, dab, daz, prebuilt);
        if (e != CSIPM_OK) return e;
        cgi += a;
        ref += b;
      }
      return CSIPM_OK;
    };
    double smu = o.sigma * mu;
    if (prebuilt) smu = c->hscal[S_SMU];   // the target the system was built for
    const double* dab = nullptr;
    const double* daz = nullptr;
    bool pred_conv = true;
    if (o.mehrotra) {
      // predictor: the affine direction (target 0), its step to the
      // boundary (at most 1) and the duality measure there,
      //   mu_a = ((1 - alpha) s.nu + alpha^2 ds.dnu) / 2n;
      // centring sigma = (mu_a / mu)^3, never aiming below the
      // complementarity the tolerance needs
      st = solve_system(0.0, nullptr, nullptr, false);
      if (st != CSIPM_OK) return st;
      pred_conv = conv;
      if (src == HD_RRES32)
        KT(c, "set_f2d", set_f2d(c->dab, c->daz, c->fxb, c->fxz, n, c->s));
      else
        KT(c, "copy_dir", copy_pair(c->dab, c->daz, c->dxb, c->dxz, n, c->s));
      KT(c, "ipm_ratio_aff+fin", ipm_step(c->beta, c->z, c->nu1, c->nu2, c->dab, c->daz, nullptr, nullptr, 0.0, 1.0,
                                          n, c->partV, c->scal, c->s, nullptr, nullptr, c->scal + S_DSDN));
      st = sync_scalars(c, "predictor");
      if (st != CSIPM_OK) return st;
      const double aa = std::min(1.0, c->hscal[S_AMAX]);
      const double nn = 2.0 * (double)n;
      const double mu_aff = std::max(0.0, ((1.0 - aa) * nn * mu + aa * aa * c->hscal[S_DSDN]) / nn);
      double sigma = std::pow(mu_aff / mu, 3.0);
      sigma = std::min(1.0, std::max(sigma, 0.1 * o.tol * (1.0 + c->xi_inf) / mu));
      smu = sigma * mu;
      dab = c->dab;
      daz = c->daz;
    }
    st = solve_system(smu, dab, daz, capture && !o.mehrotra);
    if (st != CSIPM_OK) return st;
    if (capture && !o.mehrotra && !use_learned) {
      mlp_scale_weights(c->cap_rec + (size_t)c->cap_count * c->cap_per_iter * MLP_REC, c->cap_per_iter,
                        (float)cgi, c->s);
      ++c->cap_count;
      c->cap_cg.push_back(cgi);
    }
    conv = conv && pred_conv;
    if (!conv) {
      save_state(c);
      have_snap = true;
      snap_rel = rel;
    }
    // an FP32 solution taken without refinement is read in FP32 (d = x32 exactly)
    const float* d32b = src == HD_RRES32 ? c->fxb : nullptr;
    const float* d32z = src == HD_RRES32 ? c->fxz : nullptr;
    prev_cg = cgi;
    inf.cg_iters_total += cgi;
    inf.cg_iters_max = std::max(inf.cg_iters_max, cgi);
    inf.refine_steps_total += ref;
    // The update also builds the next iteration's Newton system from the new
    // iterate (saving newton_init's pass over the state) when that system is
    // predictable: standard steps, CG, no capture, a converged solve (else
    // the next iteration recomputes G first), and in FP32 the refinement
    // expected or not from the last reduction of rel_kkt.  Its target
    // sigma mu+ comes from the step's sums.  It is built with the paper's P;
    // if the next iteration applies the learned correction, correction_patch
    // turns it into the corrected system.  A system the next iteration
    // cannot use (another precision, a recomputed G) is rebuilt by
    // newton_init.
    int fuse_kind = NEXT_NONE;
    if (o.build_next && !o.mehrotra && o.krylov == CSIPM_KRYLOV_CG && !c->cap_enable && conv && it + 1 < o.max_iter &&
        carried + 1 < kExactEvery) {
      const double rel_pred = rel * std::min(1.0, rel / prev_rel);
      if (rel_pred > o.tol) {
        if (o.precision == CSIPM_FP64) {
          fuse_kind = NEXT_F64;
        } else if (o.refine_trust > 0.0 && std::min(o.cg_rtol, 0.1 * rel_pred) >= o.refine_trust) {
          fuse_kind = NEXT_F32;
        } else if (!approx && src != HD_RRES32) {   // (after an unrefined step G is recomputed first)
          fuse_kind = NEXT_F32_REF;
        }
      }
    }
    NewtonOut<float> n32{};
    NewtonOut<double> n64{};
    NextSystem nx{nullptr, nullptr, pc_fixed};
    if (fuse_kind == NEXT_F64) {
      n64 = NewtonOut<double>{c->sig1, c->sig2, nullptr, nullptr, nullptr, nullptr,
                              c->rb, c->rz, nullptr, nullptr, c->pb, c->pz};
      nx.out64 = &n64;
    } else if (fuse_kind != NEXT_NONE) {
      const bool ref64 = fuse_kind == NEXT_F32_REF;
      n32 = NewtonOut<float>{ref64 ? c->sig1 : nullptr, ref64 ? c->sig2 : nullptr, ref64 ? c->rhb : nullptr,
                             ref64 ? c->rhz : nullptr, c->sig1f, c->sig2f, c->frb, c->frz, nullptr, nullptr,
                             c->fpb, c->fpz};
      nx.out32 = &n32;
    }
    KT(c, d32b ? "ipm_ratio_d32+fin" : "ipm_ratio+fin",
       ipm_step(c->beta, c->z, c->nu1, c->nu2, c->dxb, c->dxz, d32b, d32z, smu, o.tau, n, c->partV, c->scal, c->s,
                dab, daz, nullptr, fuse_kind != NEXT_NONE, r.csum, o.sigma));
    static const char* const kAdvName[2][4] = {
        {"ipm_advance+fin", "ipm_advance_ni32+fin", "ipm_advance_ni32r+fin", "ipm_advance_ni64+fin"},
        {"ipm_advance_d32+fin", "ipm_advance_d32_ni32+fin", "ipm_advance_d32_ni32r+fin", "ipm_advance_d32_ni64+fin"}};
    KT(c, kAdvName[d32b ? 1 : 0][fuse_kind],
       ipm_advance(c->beta, c->z, c->nu1, c->nu2, c->hb, c->dxb, c->dxz, d32b, d32z,
                   src == HD_DIRECT ? c->rb : nullptr, c->rb, src == HD_RRES32 ? c->frb : nullptr, lam, smu, c->scal, n,
                   c->partV, need_rel, c->s, dab, daz, fuse_kind != NEXT_NONE ? &nx : nullptr,
                   learned ? c->pc_act : nullptr));
    st = sync_scalars(c, "advance");
    if (st != CSIPM_OK) return st;
    r = read_resid(c);
    next_kind = fuse_kind;
    prev_rel = rel;
    exact = false;
    approx = approx || src == HD_RRES32;
    if (src == HD_RRES32) ++unrefined_steps;
    if (src == HD_RRES64) carry_err += 2.0 * DBL_EPSILON * c->hscal[S_ALPHA_IPM] * r.dscale;
    ++carried;
    c->log.push_back(csipm_iter_log{it, cgi, ref, fell ? 1 : 0, use_learned ? 1 : 0, mu, rel, 0.0, relevant});
    inf.ipm_iters = it + 1;
  }
  // (every exit of the loop above follows an FP64 recomputation of G)
  st = certificate(c, inf);
  if (st != CSIPM_OK) return st;
  inf.solve_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  inf.status = result;
  ++c->solves;
  if (info) *info = inf;
  return result;
}

csipm_status csipm_solve_batch(csipm_ctx* const* ctxs, int count, const csipm_options* opts, csipm_info* infos,
                               int* statuses, int max_threads) {
  if (count < 0 || (count > 0 && (!ctxs || !statuses))) return CSIPM_EINVAL;
  for (int i = 0; i < count; ++i) {
    if (!ctxs[i]) return CSIPM_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return CSIPM_EINVAL;
  }
  const int nt = std::max(1, std::min(count, max_threads > 0 ? max_threads : 8));
  std::atomic<int> next{0};
  auto worker = [&]() {
    for (int i = next.fetch_add(1); i < count; i = next.fetch_add(1)) {
      if (hipSetDevice(ctxs[i]->device) != hipSuccess) {
        statuses[i] = fail(ctxs[i], CSIPM_EHIP, "solve_batch: hipSetDevice");
        continue;
      }
      statuses[i] = csipm_solve(ctxs[i], opts, infos ? infos + i : nullptr);
    }
  };
  std::vector<std::thread> pool;
  pool.reserve(nt > 1 ? nt - 1 : 0);
  for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  for (int i = 0; i < count; ++i)
    if (statuses[i] < 0) return static_cast<csipm_status>(statuses[i]);
  return CSIPM_OK;
}

csipm_status csipm_get_iterate(csipm_ctx* c, int which, double* d_dst) {
  if (!c || !d_dst) return CSIPM_EINVAL;
  const double* src = nullptr;
  switch (which) {
    case CSIPM_BETA: src = c->beta; break;
    case CSIPM_Z: src = c->z; break;
    case CSIPM_NU1: src = c->nu1; break;
    case CSIPM_NU2: src = c->nu2; break;
    case CSIPM_XI: src = c->xi; break;
    case CSIPM_DIAG_H: src = c->diagH; break;
    case CSIPM_PC_C:
      launch_to_external<float, double>(c->g, c->pc_c, d_dst, c->s);
      return hip_check(c, "get_iterate");
    default: return fail(c, CSIPM_EINVAL, "unknown variable");
  }
  launch_to_external<double, double>(c->g, src, d_dst, c->s);
  return hip_check(c, "get_iterate");
}

csipm_status csipm_get_residuals(csipm_ctx* c, csipm_info* out) {
  if (!c || !out) return CSIPM_EINVAL;
  if (!c->have_lambda) return fail(c, CSIPM_ESTATE, "lambda not set");
  Resid r{};
  csipm_status st = residuals(c, r, false);
  if (st != CSIPM_OK) return st;
  std::memset(out, 0, sizeof(*out));
  out->res_beta_inf = r.fb;
  out->res_z_inf = r.fz;
  out->compl_max = r.cmax;
  out->mu = r.csum / (2.0 * (double)c->g.n);
  out->rel_kkt = std::max(std::max(r.fb, r.fz), r.cmax) / (1.0 + c->xi_inf);
  out->lambda = c->lambda;
  out->xi_inf = c->xi_inf;
  return certificate(c, *out);
}

csipm_status csipm_get_log(csipm_ctx* c, csipm_iter_log* host_buf, int max_records, int* n_records) {
  if (!c || (!host_buf && max_records > 0)) return CSIPM_EINVAL;
  const int k = std::min<int>(max_records, (int)c->log.size());
  for (int i = 0; i < k; ++i) host_buf[i] = c->log[i];
  if (n_records) *n_records = (int)c->log.size();
  return CSIPM_OK;
}

csipm_status csipm_apply_A(csipm_ctx* c, const void* d_beta, void* d_x, int precision) {
  if (!c || !d_beta || !d_x) return CSIPM_EINVAL;
  if (precision == CSIPM_FP64) {
    launch_to_internal<double, double>(c->g, (const double*)d_beta, c->pb, c->s);
    op_A<double>(c, c->pb, (double*)d_x, c->work);
  } else if (precision == CSIPM_FP32) {
    launch_to_internal<float, float>(c->g, (const float*)d_beta, c->fpb, c->s);
    op_A<float>(c, c->fpb, (float*)d_x, c->fwork);
  } else {
    return fail(c, CSIPM_EINVAL, "precision");
  }
  return hip_check(c, "apply_A");
}

csipm_status csipm_apply_At(csipm_ctx* c, const void* d_x, void* d_beta, int precision) {
  if (!c || !d_beta || !d_x) return CSIPM_EINVAL;
  if (precision == CSIPM_FP64) {
    op_At<double>(c, (const double*)d_x, c->qb, c->work);
    launch_to_external<double, double>(c->g, c->qb, (double*)d_beta, c->s);
  } else if (precision == CSIPM_FP32) {
    op_At<float>(c, (const float*)d_x, c->fqb, c->fwork);
    launch_to_external<float, float>(c->g, c->fqb, (float*)d_beta, c->s);
  } else {
    return fail(c, CSIPM_EINVAL, "precision");
  }
  return hip_check(c, "apply_At");
}

csipm_status csipm_apply_H(csipm_ctx* c, const void* d_beta, void* d_y, int precision) {
  if (!c || !d_beta || !d_y) return CSIPM_EINVAL;
  if (precision == CSIPM_FP64) {
    launch_to_internal<double, double>(c->g, (const double*)d_beta, c->pb, c->s);
    op_H<double>(c, c->pb, c->qb, c->work);
    launch_to_external<double, double>(c->g, c->qb, (double*)d_y, c->s);
  } else if (precision == CSIPM_FP32) {
    launch_to_internal<float, float>(c->g, (const float*)d_beta, c->fpb, c->s);
    op_H<float>(c, c->fpb, c->fqb, c->fwork);
    launch_to_external<float, float>(c->g, c->fqb, (float*)d_y, c->s);
  } else {
    return fail(c, CSIPM_EINVAL, "precision");
  }
  return hip_check(c, "apply_H");
}

csipm_status csipm_apply_K(csipm_ctx* c, const void* d_pb, const void* d_pz, void* d_qb, void* d_qz, int precision) {
  if (!c || !d_pb || !d_pz || !d_qb || !d_qz) return CSIPM_EINVAL;
  if (precision == CSIPM_FP64) {
    launch_to_internal<double, double>(c->g, (const double*)d_pb, c->pb, c->s);
    launch_to_internal<double, double>(c->g, (const double*)d_pz, c->pz, c->s);
    op_K<double>(c, c->pb, c->pz, c->sig1, c->sig2, c->qb, c->qz, c->work, nullptr);
    launch_to_external<double, double>(c->g, c->qb, (double*)d_qb, c->s);
    launch_to_external<double, double>(c->g, c->qz, (double*)d_qz, c->s);
  } else if (precision == CSIPM_FP32) {
    launch_to_internal<float, float>(c->g, (const float*)d_pb, c->fpb, c->s);
    launch_to_internal<float, float>(c->g, (const float*)d_pz, c->fpz, c->s);
    op_K<float>(c, c->fpb, c->fpz, c->sig1f, c->sig2f, c->fqb, c->fqz, c->fwork, nullptr);
    launch_to_external<float, float>(c->g, c->fqb, (float*)d_qb, c->s);
    launch_to_external<float, float>(c->g, c->fqz, (float*)d_qz, c->s);
  } else {
    return fail(c, CSIPM_EINVAL, "precision");
  }
  return hip_check(c, "apply_K");
}

csipm_status csipm_apply_Pinv(csipm_ctx* c, const void* d_rb, const void* d_rz, void* d_zb, void* d_zz,
                              int precision) {
  if (!c || !d_rb || !d_rz || !d_zb || !d_zz) return CSIPM_EINVAL;
  if (precision == CSIPM_FP64) {
    launch_to_internal<double, double>(c->g, (const double*)d_rb, c->rb, c->s);
    launch_to_internal<double, double>(c->g, (const double*)d_rz, c->rz, c->s);
    pinv_apply<double>(c->rb, c->rz, c->zb, c->zz, c->sig1, c->sig2, nullptr, c->g.n, c->partV, nullptr, c->s);
    launch_to_external<double, double>(c->g, c->zb, (double*)d_zb, c->s);
    launch_to_external<double, double>(c->g, c->zz, (double*)d_zz, c->s);
  } else if (precision == CSIPM_FP32) {
    launch_to_internal<float, float>(c->g, (const float*)d_rb, c->frb, c->s);
    launch_to_internal<float, float>(c->g, (const float*)d_rz, c->frz, c->s);
    pinv_apply<float>(c->frb, c->frz, c->fzb, c->fzz, c->sig1f, c->sig2f, nullptr, c->g.n, c->partV, nullptr,
                      c->s);
    launch_to_external<float, float>(c->g, c->fzb, (float*)d_zb, c->s);
    launch_to_external<float, float>(c->g, c->fzz, (float*)d_zz, c->s);
  } else {
    return fail(c, CSIPM_EINVAL, "precision");
  }
  return hip_check(c, "apply_Pinv");
}

csipm_status csipm_set_barrier(csipm_ctx* c, const double* d_sigma1, const double* d_sigma2) {
  if (!c || !d_sigma1 || !d_sigma2) return CSIPM_EINVAL;
  launch_to_internal<double, double>(c->g, d_sigma1, c->sig1, c->s);
  launch_to_internal<double, double>(c->g, d_sigma2, c->sig2, c->s);
  launch_to_internal<double, float>(c->g, d_sigma1, c->sig1f, c->s);
  launch_to_internal<double, float>(c->g, d_sigma2, c->sig2f, c->s);
  if (c->g.n > c->g.nr) {   // the coordinate without data keeps Sigma = 1 (P stays invertible there)
    fill<double>(c->sig1 + c->g.nr, 1.0, 1, c->s);
    fill<double>(c->sig2 + c->g.nr, 1.0, 1, c->s);
    fill<float>(c->sig1f + c->g.nr, 1.0f, 1, c->s);
    fill<float>(c->sig2f + c->g.nr, 1.0f, 1, c->s);
  }
  return hip_check(c, "set_barrier");
}

csipm_status csipm_set_pc_params(csipm_ctx* c, const float* d_params, int n_params) {
  if (!c || !d_params) return CSIPM_EINVAL;
  if (n_params != CSIPM_MLP_PARAMS) return fail(c, CSIPM_EINVAL, "expected 1249 parameters");
  hipError_t e = hipMemcpyAsync(c->mlp_params, d_params, sizeof(float) * MLP_NP, hipMemcpyDeviceToDevice, c->s);
  if (e != hipSuccess) return fail(c, CSIPM_EHIP, hipGetErrorString(e));
  c->have_params = true;
  return CSIPM_OK;
}

size_t csipm_mlp_scratch_bytes(int n_rec) {
  if (n_rec < 0) return 0;
  const size_t nblk = ((size_t)n_rec + 63) / 64;
  return std::max<size_t>(1, nblk) * (MLP_NP + 1) * sizeof(double);
}

csipm_status csipm_mlp_forward(const float* d_params, const float* d_feat, float* d_c, int n_rec, void* hip_stream) {
  if (!d_params || !d_feat || !d_c || n_rec < 0) return CSIPM_EINVAL;
  if (n_rec == 0) return CSIPM_OK;
  mlp_forward(d_params, d_feat, d_c, n_rec, reinterpret_cast<hipStream_t>(hip_stream));
  return hipGetLastError() == hipSuccess ? CSIPM_OK : CSIPM_EHIP;
}

csipm_status csipm_mlp_backward(const float* d_params, const float* d_feat, const float* d_dc, float* d_grad,
                                int n_rec, void* d_scratch, size_t scratch_bytes, void* hip_stream) {
  if (!d_params || !d_feat || !d_dc || !d_grad || !d_scratch || n_rec < 0) return CSIPM_EINVAL;
  if (scratch_bytes < csipm_mlp_scratch_bytes(n_rec)) return CSIPM_ENOMEM;
  if (n_rec == 0) return CSIPM_OK;
  mlp_backward(d_params, d_feat, d_dc, d_grad, n_rec, (double*)d_scratch, reinterpret_cast<hipStream_t>(hip_stream));
  return hipGetLastError() == hipSuccess ? CSIPM_OK : CSIPM_EHIP;
}

csipm_status csipm_mlp_loss_grad(const float* d_params, const float* d_feat, const float* d_rec, int n_rec,
                                 double* d_loss_out, float* d_grad, void* d_scratch, size_t scratch_bytes,
                                 void* hip_stream) {
  if (!d_params || !d_feat || !d_rec || !d_loss_out || !d_grad || !d_scratch || n_rec < 1) return CSIPM_EINVAL;
  if (scratch_bytes < csipm_mlp_scratch_bytes(n_rec)) return CSIPM_ENOMEM;
  mlp_loss_grad(d_params, d_feat, d_rec, n_rec, d_loss_out, d_grad, (double*)d_scratch,
                reinterpret_cast<hipStream_t>(hip_stream));
  return hipGetLastError() == hipSuccess ? CSIPM_OK : CSIPM_EHIP;
}

csipm_status csipm_mlp_adam(float* d_params, const float* d_grad, float* d_m, float* d_v, int t, float lr,
                            void* hip_stream) {
  if (!d_params || !d_grad || !d_m || !d_v || t < 1 || !(lr > 0.0f)) return CSIPM_EINVAL;
  mlp_adam(d_params, d_grad, d_m, d_v, t, lr, reinterpret_cast<hipStream_t>(hip_stream));
  return hipGetLastError() == hipSuccess ? CSIPM_OK : CSIPM_EHIP;
}

csipm_status csipm_mlp_train_step(float* d_params, float* d_m, float* d_v, int t, float lr, const float* d_feat,
                                  const float* d_rec, int n_rec, double* d_loss_out, float* d_grad, void* d_scratch,
                                  size_t scratch_bytes, void* hip_stream) {
  if (!d_params || !d_m || !d_v || t < 1 || !(lr > 0.0f)) return CSIPM_EINVAL;
  const csipm_status st =
      csipm_mlp_loss_grad(d_params, d_feat, d_rec, n_rec, d_loss_out, d_grad, d_scratch, scratch_bytes, hip_stream);
  if (st != CSIPM_OK) return st;
  return csipm_mlp_adam(d_params, d_grad, d_m, d_v, t, lr, hip_stream);
}

csipm_status csipm_capture(csipm_ctx* c, int enable, float* d_feat, float* d_rec, int n_per_iter, int max_iters,
                           unsigned long long seed) {
  if (!c) return CSIPM_EINVAL;
  if (!enable) {
    c->cap_enable = 0;
    return CSIPM_OK;
  }
  if (!d_feat || !d_rec || n_per_iter < 1 || max_iters < 1) return fail(c, CSIPM_EINVAL, "capture buffers");
  if (enable != 1 && enable != 2) return fail(c, CSIPM_EINVAL, "capture mode");
  c->cap_enable = enable;
  c->cap_feat = d_feat;
  c->cap_rec = d_rec;
  c->cap_per_iter = n_per_iter;
  c->cap_max = max_iters;
  c->cap_seed = seed;
  c->cap_count = 0;
  c->cap_cg.clear();
  return CSIPM_OK;
}

csipm_status csipm_captured(csipm_ctx* c, int* n_iters, int* cg_counts_host, int max_iters) {
  if (!c) return CSIPM_EINVAL;
  if (n_iters) *n_iters = c->cap_count;
  if (cg_counts_host)
    for (int i = 0; i < std::min<int>(max_iters, (int)c->cap_cg.size()); ++i) cg_counts_host[i] = c->cap_cg[i];
  return CSIPM_OK;
}

csipm_status csipm_pc_correction(csipm_ctx* c, double* d_c) {
  if (!c || !d_c) return CSIPM_EINVAL;
  if (!c->have_params) return fail(c, CSIPM_ESTATE, "learned preconditioner has no parameters");
  absmax(c->beta, c->g.n, c->partV, c->scal + S_RESID + 4, c->s);
  csipm_status st = learned_correction(c, false);
  if (st != CSIPM_OK) return st;
  launch_to_external<float, double>(c->g, c->pc_c, d_c, c->s);
  return hip_check(c, "pc_correction");
}

csipm_status csipm_features(csipm_ctx* c, float* d_feat) {
  if (!c || !d_feat) return CSIPM_EINVAL;
  absmax(c->beta, c->g.n, c->partV, c->scal + S_RESID + 4, c->s);
  compute_features(c);
  launch_feat_to_external(c->g, c->feat, d_feat, c->s);
  return hip_check(c, "features");
}

csipm_status csipm_profile_kapply(csipm_ctx* c, int precision, int reps, double* ms_out) {
  if (!c || !ms_out || reps < 1) return CSIPM_EINVAL;
  if (precision != CSIPM_FP64 && precision != CSIPM_FP32) return fail(c, CSIPM_EINVAL, "precision");
  const Grid& g = c->g;
  if (g.odd3()) return fail(c, CSIPM_EUNSUPPORTED, "profile_kapply: the five-pass K-apply needs an even N3");
  hipEvent_t ev[CSIPM_KAPPLY_PASSES + 1];
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) return fail(c, CSIPM_EHIP, "hipEventCreate");
  double acc[CSIPM_KAPPLY_PASSES] = {0};
  double whole = 0.0, direct = 0.0;
  auto run = [&](auto tag) {
    using T = decltype(tag);
    PcgSet v = pcg_set<T>(c);
    T *pb = (T*)v.pb, *pz = (T*)v.pz, *qb = (T*)v.qb, *qz = (T*)v.qz, *work = (T*)v.work;
    const T* s1 = std::is_same<T, double>::value ? (const T*)c->sig1 : (const T*)c->sig1f;
    const T* s2 = std::is_same<T, double>::value ? (const T*)c->sig2 : (const T*)c->sig2f;
    const int ps = (int)k_partials(g.n1, g.n2, g.n3);
    EpiArgs<T> ka{KArgs<T>{pb, pz, s1, s2, qb, qz, PUpd<T>{}}, RArgs{}, c->partK, ps};
    for (int r = 0; r < reps; ++r) {
      (void)hipEventRecord(ev[0], c->s);
      launch_axis12<T>(g, 1, +1, pb, work, tw<T>(c), EPI_NONE, nullptr, nullptr, c->s);
      (void)hipEventRecord(ev[1], c->s);
      launch_axis12<T>(g, 2, +1, work, work, tw<T>(c), EPI_NONE, nullptr, nullptr, c->s);
      (void)hipEventRecord(ev[2], c->s);
      launch_axis3<T>(g, A3_FULL, work, work, c->mask, tw<T>(c), nullptr, c->s);
      (void)hipEventRecord(ev[3], c->s);
      launch_axis12<T>(g, 2, -1, work, work, tw<T>(c), EPI_NONE, nullptr, nullptr, c->s);
      (void)hipEventRecord(ev[4], c->s);
      launch_axis12<T>(g, 1, -1, work, work, tw<T>(c), EPI_K, &ka, nullptr, c->s);
      (void)hipEventRecord(ev[5], c->s);
      (void)hipEventSynchronize(ev[5]);
      for (int k = 0; k < CSIPM_KAPPLY_PASSES; ++k) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
        acc[k] += ms;
      }
    }
    // the same K-apply back to back, one event pair around all reps:
    // launched directly, and replayed from a HIP graph of the reps applies
    // (as a solve launches its PCG iterations)
    (void)hipEventRecord(ev[0], c->s);
    for (int r = 0; r < reps; ++r) (void)op_K<T>(c, pb, pz, s1, s2, qb, qz, work, nullptr);
    (void)hipEventRecord(ev[1], c->s);
    (void)hipEventSynchronize(ev[1]);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
    direct = (double)ms / reps;
    whole = direct;
    if (!c->cap_s && hipStreamCreateWithFlags(&c->cap_s, hipStreamNonBlocking) != hipSuccess) c->cap_s = nullptr;
    if (c->cap_s) {
      hipStream_t s0 = c->s;
      c->s = c->cap_s;
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      bool ok = hipStreamBeginCapture(c->cap_s, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        for (int r = 0; r < reps; ++r) (void)op_K<T>(c, pb, pz, s1, s2, qb, qz, work, nullptr);
        ok = hipStreamEndCapture(c->cap_s, &graph) == hipSuccess && graph;
      }
      c->s = s0;
      if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
      if (graph) (void)hipGraphDestroy(graph);
      if (ok) {
        (void)hipGraphLaunch(exec, c->s);   // (first replay uploads the graph)
        (void)hipEventRecord(ev[0], c->s);
        (void)hipGraphLaunch(exec, c->s);
        (void)hipEventRecord(ev[1], c->s);
        (void)hipEventSynchronize(ev[1]);
        ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
        whole = (double)ms / reps;
      } else {
        (void)hipGetLastError();
      }
      if (exec) (void)hipGraphExecDestroy(exec);
    }
  };
  if (precision == CSIPM_FP64) run(double{}); else run(float{});
  for (auto& e : ev) (void)hipEventDestroy(e);
  for (int k = 0; k < CSIPM_KAPPLY_PASSES; ++k) ms_out[k] = acc[k] / reps;
  ms_out[CSIPM_KAPPLY_PASSES] = whole;
  ms_out[CSIPM_KAPPLY_PASSES + 1] = direct;
  return hip_check(c, "profile_kapply");
}

csipm_status csipm_timing(csipm_ctx* c, int enable) {
  if (!c) return CSIPM_EINVAL;
  if (enable) {
    c->kt_rec.clear();
    c->kt_dropped = 0;
  }
  c->kt_on = enable != 0;
  return CSIPM_OK;
}

csipm_status csipm_timing_report(csipm_ctx* c, double min_us, csipm_kernel_time* out, int max_records,
                                 int* n_records) {
  if (!c || (!out && max_records > 0)) return CSIPM_EINVAL;
  hipError_t e = hipStreamSynchronize(c->s);
  if (e != hipSuccess) return fail(c, CSIPM_EHIP, std::string("timing_report: ") + hipGetErrorString(e));
  std::vector<csipm_kernel_time> agg;
  for (const auto& rec : c->kt_rec) {
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, c->kt_ev[rec.second], c->kt_ev[rec.second + 1]);
    if (e != hipSuccess) return fail(c, CSIPM_EHIP, std::string("timing_report: ") + hipGetErrorString(e));
    size_t k = 0;
    while (k < agg.size() && std::strcmp(agg[k].name, rec.first) != 0) ++k;
    if (k == agg.size()) {
      csipm_kernel_time t{};
      std::snprintf(t.name, sizeof(t.name), "%s", rec.first);
      agg.push_back(t);
    }
    agg[k].calls += 1;
    agg[k].total_ms += ms;
    if (ms * 1e3 >= min_us) {
      agg[k].working_calls += 1;
      agg[k].working_ms += ms;
    }
  }
  if (!agg.empty()) agg[0].dropped = c->kt_dropped;
  for (int i = 0; i < std::min<int>(max_records, (int)agg.size()); ++i) out[i] = agg[i];
  if (n_records) *n_records = (int)agg.size();
  return CSIPM_OK;
}

csipm_status csipm_destroy(csipm_ctx* c) {
  if (!c) return CSIPM_EINVAL;
  for (hipEvent_t ev : c->kt_ev) (void)hipEventDestroy(ev);
  for (auto& gr : c->graphs) (void)hipGraphExecDestroy(gr.exec);
  if (c->cap_s) (void)hipStreamDestroy(c->cap_s);
  if (c->hscal) (void)hipHostFree(c->hscal);
  delete c;
  return CSIPM_OK;
}

const char* csipm_status_string(int st) {
  switch (st) {
    case CSIPM_OK: return "ok";
    case CSIPM_NOT_CONVERGED: return "not converged (iteration limit)";
    case CSIPM_STALLED: return "stalled (step length collapsed)";
    case CSIPM_FELL_BACK: return "converged with preconditioner fallbacks";
    case CSIPM_EINVAL: return "invalid argument";
    case CSIPM_ENOMEM: return "workspace too small";
    case CSIPM_EHIP: return "HIP runtime error";
    case CSIPM_ENONFINITE: return "non-finite value";
    case CSIPM_EUNSUPPORTED: return "unsupported grid";
    case CSIPM_ESTATE: return "call out of order";
  }
  return "unknown status";
}

const char* csipm_last_error(const csipm_ctx* c) { return c ? c->err.c_str() : noctx_last_error(); }

}  // extern "C"
