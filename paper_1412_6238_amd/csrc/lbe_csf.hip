// lbe_csf.hip -- host side of liblbe_csf.so: parameter checks, workspace
// layout, launch configuration and the C ABI declared in include/lbe_csf.h.
//
// The library owns no device memory: every buffer is carved out of the
// caller's workspace.  Layout (each region 256-byte aligned):
//   state A, state B     row-interleaved: per row, 25 plane segments (FP64, or
//                        FP32 deviations), g_0 (FP64) and hbar_0 (FP64, or an
//                        FP32 deviation)
//   wall temperatures    2 * nx FP64 (bottom, top)
//   partials             max blocks * 7 FP64 (per-block diagnostic sums)
//   diag ring            4096 records of (step, 7 sums)
//   counters             records written, non-finite total
//   one record           target of synchronous diagnostics
//   pressure plane       nx * ny FP64, with two densities only (Eq. 9)
//   adjoint region       present when record_steps > 0 (see adjoint.h)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbe_csf.h"
#include "adjoint.h"
#include "aux_kernels.h"
#include "step_kernel.h"

using namespace lbe;
using namespace lbe::host;

namespace {

thread_local std::string g_create_error;

}  // namespace

struct lbe_csf {
  lbe_csf_params P;
  Layout L;
  Launch la;
  hipStream_t stream;
  char *ws;
  void *state[2];
  int cur;
  int64_t step;
  double *tw;         // [2][nx]
  double *partials;
  DiagRecord *ring;
  int64_t *counters;
  DiagRecord *rec;    // one record for synchronous diagnostics
  int64_t record_cap;
  // record of the last recorded run
  bool recorded;
  int64_t rec_start, rec_steps, rec_K;
  std::string err;
  StepArgs base;      // constants filled once
  int device;         // the HIP device current at creation
  bool tile;          // steps in tiles (tile_step_kernel; latency-bound grids)
  int diag_blocks;    // diagnostic partials per launch (blocks of the step kernel used)
  size_t small_lds;   // > 0: plain steps run many per launch (small grids)
  bool small_res;     // ... with both states resident in LDS
  hipStream_t aux = nullptr;   // second stream of the backward pass (made on first use)
  ~lbe_csf() {
    if (aux) {
      int prev = 0;
      if (hipGetDevice(&prev) == hipSuccess && prev != device) (void)hipSetDevice(device);
      (void)hipStreamDestroy(aux);
      if (prev != device) (void)hipSetDevice(prev);
    }
  }
};

namespace {

int fail(lbe_csf *h, int code, const std::string &msg) {
  if (h) h->err = msg;
  else g_create_error = msg;
  return code;
}

#define HIPCHK(h, expr)                                                        \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess)                                                      \
      return fail(h, LBE_CSF_EDEVICE,                                          \
                  std::string(#expr) + ": " + hipGetErrorString(e_));          \
  } while (0)

void fill_constants(lbe_csf *h) {
  const lbe_csf_params &p = h->P;
  StepArgs &a = h->base;
  std::memset(&a, 0, sizeof(a));
  a.nx = p.nx;
  a.ny = p.ny;
  a.walls_y = p.walls_y;
  a.nstrips = h->la.nstrips;
  a.rows_per_chunk = h->la.rows;
  a.twb = h->tw;
  a.twt = h->tw + p.nx;
  a.rho = p.rho;
  a.cv = p.cv;
  a.rcv = p.rho * p.cv;
  a.drho = two_densities(&p) ? p.rho2 - p.rho : 0.0;
  a.pc = two_densities(&p) ? reinterpret_cast<const double *>(h->ws + h->L.off_pc) : nullptr;
  a.pc_out = two_densities(&p) ? reinterpret_cast<double *>(h->ws + h->L.off_pc) : nullptr;
  a.tauf0 = p.tau_f[0];
  a.dtauf = p.tau_f[1] - p.tau_f[0];
  a.tauT0 = p.tau_T[0];
  a.dtauT = p.tau_T[1] - p.tau_T[0];
  a.omg_g = 1.0 / p.tau_g;
  // interface constants: W is the tanh denominator of the planar profile,
  // eps = W sqrt(beta/2); alpha = 3 sqrt(2/beta) makes eps alpha int c'^2 = 1
  const double eps = p.width * std::sqrt(p.beta / 2.0);
  const double alpha = 3.0 * std::sqrt(2.0 / p.beta);
  const double Gamma = p.mobility / (p.tau_g - 0.5);
  a.gam3 = 3.0 * Gamma;
  a.beta2 = 2.0 * p.beta;
  a.eps2 = eps * eps;
  a.kcap = alpha / eps;
  a.epsalpha = eps * alpha;
  a.sigma0 = p.sigma0;
  a.sigmaT = p.sigmaT;
  a.Tref = p.Tref;
  a.ax = p.force[0];
  a.ay = p.force[1];
  a.p0 = p.precision == LBE_CSF_FP32_DEV ? p.p0 : 0.0;
  a.Ts = p.precision == LBE_CSF_FP32_DEV ? p.T_shift : 0.0;
  a.Tg = p.precision == LBE_CSF_FP32_DEV ? p.T_grad : 0.0;
  a.partials = h->partials;
}

template <typename S, typename R, bool DEV, int MODE, int PIPE>
void launch_pipe(const Launch &la, const StepArgs &a, hipStream_t st) {
  switch (la.nw) {
    case 1: step_kernel<S, R, DEV, MODE, 1, PIPE><<<la.nblocks, 64, 0, st>>>(a); break;
    case 2: step_kernel<S, R, DEV, MODE, 2, PIPE><<<la.nblocks, 128, 0, st>>>(a); break;
    case 8: step_kernel<S, R, DEV, MODE, 8, PIPE><<<la.nblocks, 512, 0, st>>>(a); break;
    default: step_kernel<S, R, DEV, MODE, 4, PIPE><<<la.nblocks, 256, 0, st>>>(a); break;
  }
}

template <typename S, typename R, bool DEV, int MODE>
void launch_mode(const Launch &la, const StepArgs &a, hipStream_t st) {
  if constexpr ((MODE & kVarRho) != 0) {
    launch_pipe<S, R, DEV, MODE, 1>(la, a, st);   // two densities: rows one ahead
  } else {
    switch (la.pipe) {
      case 0: launch_pipe<S, R, DEV, MODE, 0>(la, a, st); break;
      case 2: launch_pipe<S, R, DEV, MODE, 2>(la, a, st); break;
      default: launch_pipe<S, R, DEV, MODE, 1>(la, a, st); break;
    }
  }
}

// Launch the step kernel instantiated for this mode; false (nothing
// launched) for a combination of mode bits that has no instantiation.
template <typename S, typename R, bool DEV>
bool launch_prec(int mode, const Launch &la, const StepArgs &a, hipStream_t st) {
  switch (mode) {
    case kStore: launch_mode<S, R, DEV, kStore>(la, a, st); return true;
    case kStore | kDiag: launch_mode<S, R, DEV, kStore | kDiag>(la, a, st); return true;
    case kFields: launch_mode<S, R, DEV, kFields>(la, a, st); return true;
    case kDiag: launch_mode<S, R, DEV, kDiag>(la, a, st); return true;
    case kStore | kTape: launch_mode<S, R, DEV, kStore | kTape>(la, a, st); return true;
    case kTape: launch_mode<S, R, DEV, kTape>(la, a, st); return true;
    case kStore | kCurv: launch_mode<S, R, DEV, kStore | kCurv>(la, a, st); return true;
    case kStore | kDiag | kCurv: launch_mode<S, R, DEV, kStore | kDiag | kCurv>(la, a, st); return true;
    case kFields | kCurv: launch_mode<S, R, DEV, kFields | kCurv>(la, a, st); return true;
    case kDiag | kCurv: launch_mode<S, R, DEV, kDiag | kCurv>(la, a, st); return true;
    case kStore | kTape | kCurv: launch_mode<S, R, DEV, kStore | kTape | kCurv>(la, a, st); return true;
    case kTape | kCurv: launch_mode<S, R, DEV, kTape | kCurv>(la, a, st); return true;
    default: break;
  }
  if constexpr (DEV) {
    // whole-line stores past the last-level cache (FP32 form, one density)
    constexpr int T = kStream;
    switch (mode) {
      case kStore | T: launch_mode<S, R, DEV, kStore | T>(la, a, st); return true;
      case kStore | kDiag | T: launch_mode<S, R, DEV, kStore | kDiag | T>(la, a, st); return true;
      case kStore | kCurv | T: launch_mode<S, R, DEV, kStore | kCurv | T>(la, a, st); return true;
      case kStore | kDiag | kCurv | T:
        launch_mode<S, R, DEV, kStore | kDiag | kCurv | T>(la, a, st); return true;
      default: break;
    }
  }
  // two densities: the pressure pass, then the step
  constexpr int V = kVarRho, P = kVarRho | kPress;
  switch (mode) {
    case P: launch_mode<S, R, DEV, P>(la, a, st); return true;
    case P | kCurv: launch_mode<S, R, DEV, P | kCurv>(la, a, st); return true;
    case V | kStore: launch_mode<S, R, DEV, V | kStore>(la, a, st); return true;
    case V | kStore | kDiag: launch_mode<S, R, DEV, V | kStore | kDiag>(la, a, st); return true;
    case V | kFields: launch_mode<S, R, DEV, V | kFields>(la, a, st); return true;
    case V | kDiag: launch_mode<S, R, DEV, V | kDiag>(la, a, st); return true;
    case V | kStore | kCurv: launch_mode<S, R, DEV, V | kStore | kCurv>(la, a, st); return true;
    case V | kStore | kDiag | kCurv:
      launch_mode<S, R, DEV, V | kStore | kDiag | kCurv>(la, a, st); return true;
    case V | kFields | kCurv: launch_mode<S, R, DEV, V | kFields | kCurv>(la, a, st); return true;
    case V | kDiag | kCurv: launch_mode<S, R, DEV, V | kDiag | kCurv>(la, a, st); return true;
    default: return false;
  }
}

bool launch_any(bool f64, int mode, const Launch &la, const StepArgs &a, hipStream_t st) {
  return f64 ? launch_prec<double, double, false>(mode, la, a, st)
             : launch_prec<float, float, true>(mode, la, a, st);
}

// The tile kernel instantiated for this mode; false for a mode without one.
template <typename S, typename R, bool DEV>
bool launch_tile(int mode, int nb, const StepArgs &a, hipStream_t st) {
  constexpr int T = kTileX * kTileY;
  switch (mode) {
    case kStore: tile_step_kernel<S, R, DEV, kStore><<<nb, T, 0, st>>>(a); return true;
    case kStore | kDiag: tile_step_kernel<S, R, DEV, kStore | kDiag><<<nb, T, 0, st>>>(a); return true;
    case kFields: tile_step_kernel<S, R, DEV, kFields><<<nb, T, 0, st>>>(a); return true;
    case kDiag: tile_step_kernel<S, R, DEV, kDiag><<<nb, T, 0, st>>>(a); return true;
    case kStore | kTape: tile_step_kernel<S, R, DEV, kStore | kTape><<<nb, T, 0, st>>>(a); return true;
    case kTape: tile_step_kernel<S, R, DEV, kTape><<<nb, T, 0, st>>>(a); return true;
    case kStore | kCurv: tile_step_kernel<S, R, DEV, kStore | kCurv><<<nb, T, 0, st>>>(a); return true;
    case kStore | kDiag | kCurv:
      tile_step_kernel<S, R, DEV, kStore | kDiag | kCurv><<<nb, T, 0, st>>>(a); return true;
    case kFields | kCurv: tile_step_kernel<S, R, DEV, kFields | kCurv><<<nb, T, 0, st>>>(a); return true;
    case kDiag | kCurv: tile_step_kernel<S, R, DEV, kDiag | kCurv><<<nb, T, 0, st>>>(a); return true;
    case kStore | kTape | kCurv:
      tile_step_kernel<S, R, DEV, kStore | kTape | kCurv><<<nb, T, 0, st>>>(a); return true;
    case kTape | kCurv: tile_step_kernel<S, R, DEV, kTape | kCurv><<<nb, T, 0, st>>>(a); return true;
    default: break;
  }
  // two densities: the pressure pass, then the step
  constexpr int V = kVarRho, P = kVarRho | kPress;
  switch (mode) {
    case P: tile_step_kernel<S, R, DEV, P><<<nb, T, 0, st>>>(a); return true;
    case P | kCurv: tile_step_kernel<S, R, DEV, P | kCurv><<<nb, T, 0, st>>>(a); return true;
    case V | kStore: tile_step_kernel<S, R, DEV, V | kStore><<<nb, T, 0, st>>>(a); return true;
    case V | kStore | kDiag: tile_step_kernel<S, R, DEV, V | kStore | kDiag><<<nb, T, 0, st>>>(a); return true;
    case V | kFields: tile_step_kernel<S, R, DEV, V | kFields><<<nb, T, 0, st>>>(a); return true;
    case V | kDiag: tile_step_kernel<S, R, DEV, V | kDiag><<<nb, T, 0, st>>>(a); return true;
    case V | kStore | kCurv: tile_step_kernel<S, R, DEV, V | kStore | kCurv><<<nb, T, 0, st>>>(a); return true;
    case V | kStore | kDiag | kCurv:
      tile_step_kernel<S, R, DEV, V | kStore | kDiag | kCurv><<<nb, T, 0, st>>>(a); return true;
    case V | kFields | kCurv: tile_step_kernel<S, R, DEV, V | kFields | kCurv><<<nb, T, 0, st>>>(a); return true;
    case V | kDiag | kCurv: tile_step_kernel<S, R, DEV, V | kDiag | kCurv><<<nb, T, 0, st>>>(a); return true;
    default: return false;
  }
}

int launch_step_on(lbe_csf *h, hipStream_t stream, int mode, const void *src, void *dst,
                   double *phi, double *ux, double *uy, double *p, double *T,
                   void *tape = nullptr, double *partials = nullptr) {
  StepArgs a = h->base;
  if (partials) a.partials = partials;
  a.src = src;
  a.dst = dst;
  a.tape = tape;
  a.phi = phi;
  a.ux = ux;
  a.uy = uy;
  a.p = p;
  a.T = T;
  if (h->P.csf_form == 1) mode |= kCurv;
  if (h->la.stream && (mode & kStore) && !(mode & kTape)) mode |= kStream;
  if (h->tile) {
    // latency-bound grid: the step in tiles (tile_step_kernel); with two
    // densities the pressure pass first, as below
    const int nb = tile_blocks(h->P.nx, h->P.ny);
    const bool f64 = h->P.precision == LBE_CSF_FP64;
    int tm = mode & ~kStream;
    if (a.drho != 0.0) {
      const int pm = kVarRho | kPress | (tm & kCurv);
      if (!(f64 ? launch_tile<double, double, false>(pm, nb, a, stream)
                : launch_tile<float, float, true>(pm, nb, a, stream)))
        return fail(h, LBE_CSF_EINVAL, "no tile kernel for mode " + std::to_string(pm));
      HIPCHK(h, hipGetLastError());
      tm |= kVarRho;
    }
    if (!(f64 ? launch_tile<double, double, false>(tm, nb, a, stream)
              : launch_tile<float, float, true>(tm, nb, a, stream)))
      return fail(h, LBE_CSF_EINVAL, "no tile kernel for mode " + std::to_string(tm));
    HIPCHK(h, hipGetLastError());
    return LBE_CSF_OK;
  }
  if (a.drho != 0.0) {
    // two densities: the pressure of Eq. 9 of the source state first (it
    // needs u, hence the force, at every site of the stencil)
    const int pm = kVarRho | kPress | (mode & kCurv);
    if (!launch_any(h->P.precision == LBE_CSF_FP64, pm, h->la, a, stream))
      return fail(h, LBE_CSF_EINVAL, "no step kernel for mode " + std::to_string(pm));
    HIPCHK(h, hipGetLastError());
    mode |= kVarRho;
  }
  if (!launch_any(h->P.precision == LBE_CSF_FP64, mode, h->la, a, stream))
    return fail(h, LBE_CSF_EINVAL, "no step kernel for mode " + std::to_string(mode));
  HIPCHK(h, hipGetLastError());
  return LBE_CSF_OK;
}

int launch_step(lbe_csf *h, int mode, const void *src, void *dst, double *phi, double *ux,
                double *uy, double *p, double *T, void *tape = nullptr,
                double *partials = nullptr) {
  return launch_step_on(h, h->stream, mode, src, dst, phi, ux, uy, p, T, tape, partials);
}

// Plain steps of a small grid, up to kSmallRun per launch of one block
// (small_step_kernel); the states alternate as with one launch per step.
constexpr int64_t kSmallRun = 4096;
template <typename S, typename R, bool DEV, int MODE, bool RES>
hipError_t small_attr(size_t lds) {
  return hipFuncSetAttribute(
      reinterpret_cast<const void *>(&small_step_kernel<S, R, DEV, MODE, RES>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}
template <typename S, typename R, bool DEV, bool RES>
hipError_t small_attrs(size_t lds) {
  hipError_t e = small_attr<S, R, DEV, kStore, RES>(lds);
  if (e == hipSuccess) e = small_attr<S, R, DEV, kStore | kCurv, RES>(lds);
  return e;
}
template <typename S, typename R, bool DEV, int MODE>
void small_launch(const StepArgs &a, void *other, int steps, int threads, size_t lds, bool res,
                  hipStream_t st) {
  if (res) small_step_kernel<S, R, DEV, MODE, true><<<1, threads, lds, st>>>(a, other, steps);
  else small_step_kernel<S, R, DEV, MODE, false><<<1, threads, lds, st>>>(a, other, steps);
}

int launch_small(lbe_csf *h, int64_t nsteps) {
  const size_t n = (size_t)h->P.nx * h->P.ny;
  const int threads = (int)std::min<size_t>(kSmallMaxSites, (n + 63) / 64 * 64);
  const bool f64 = h->P.precision == LBE_CSF_FP64, curv = h->P.csf_form == 1;
  while (nsteps > 0) {
    const int m = (int)std::min(nsteps, kSmallRun);
    StepArgs a = h->base;
    a.src = h->state[h->cur];
    void *other = h->state[1 - h->cur];
    const size_t lds = h->small_lds;
    const bool res = h->small_res;
    if (f64 && !curv) small_launch<double, double, false, kStore>(a, other, m, threads, lds, res, h->stream);
    else if (f64) small_launch<double, double, false, kStore | kCurv>(a, other, m, threads, lds, res, h->stream);
    else if (!curv) small_launch<float, float, true, kStore>(a, other, m, threads, lds, res, h->stream);
    else small_launch<float, float, true, kStore | kCurv>(a, other, m, threads, lds, res, h->stream);
    HIPCHK(h, hipGetLastError());
    if (m & 1) h->cur = 1 - h->cur;
    h->step += m;
    nsteps -= m;
  }
  return LBE_CSF_OK;
}

int launch_reduce(lbe_csf *h, int64_t step, bool append) {
  if (append)
    diag_reduce_kernel<<<1, 256, 0, h->stream>>>(h->partials, h->diag_blocks, h->ring,
                                                 kDiagRing, h->counters, step);
  else
    diag_reduce_kernel<<<1, 256, 0, h->stream>>>(h->partials, h->diag_blocks, h->rec, 1,
                                                 nullptr, step);
  HIPCHK(h, hipGetLastError());
  return LBE_CSF_OK;
}

// One adjoint step: collision transpose, then stencil transpose.
template <typename R, bool DEV, bool CURV>
void launch_adj(bool vartau, const AdjArgs &aa, int nblocks, hipStream_t st) {
  if (vartau) adj_collide_kernel<R, DEV, true, CURV><<<nblocks, kAdjTX * kAdjTY, 0, st>>>(aa);
  else adj_collide_kernel<R, DEV, false, CURV><<<nblocks, kAdjTX * kAdjTY, 0, st>>>(aa);
  adj_stencil_kernel<R, CURV><<<nblocks, kAdjTX * kAdjTY, 0, st>>>(aa);
}

// Reverse sweep over the recorded run: for each segment, last first, replay
// the forward steps from its checkpoint (writing the moment tape, and keeping
// the states when the relaxation times vary with c), then apply the adjoint
// step in reverse order.
int run_backward(lbe_csf *h, const double *dJdc, double *dsT, double *dTw, double *dF0,
                 double *dT0) {
  const AdjLayout &A = h->L.adj;
  char *base = h->ws + h->L.off_adj;
  const int nx = h->P.nx, ny = h->P.ny;
  const size_t n = (size_t)nx * ny;
  const bool f64 = h->P.precision == LBE_CSF_FP64;
  hipStream_t st = h->stream;
  char *lam = base + A.off_lam;
  const size_t pl = A.plane_bytes;
  void *D[2] = {lam, lam + 27 * pl};
  void *M[2] = {lam + 54 * pl, lam + 57 * pl};
  void *Abuf = lam + 60 * pl;
  double *part = reinterpret_cast<double *>(base + A.off_part);
  double *tw = reinterpret_cast<double *>(base + A.off_tw);
  double *outv = reinterpret_cast<double *>(base + A.off_out);
  const int ntx = adj_tiles_x(nx), nb = ntx * adj_tiles_y(ny);
  adj_zero_kernel<<<(nb + 255) / 256, 256, 0, st>>>(part, (size_t)nb);
  adj_zero_kernel<<<(2 * nx + 255) / 256, 256, 0, st>>>(tw, 2 * (size_t)nx);
  const dim3 g27((unsigned)((n + 255) / 256), 27);
  if (f64)
    adj_seed_kernel<double><<<g27, 256, 0, st>>>(static_cast<double *>(D[0]),
                                                 static_cast<double *>(M[0]), dJdc, n,
                                                 (size_t)nx);
  else
    adj_seed_kernel<float><<<g27, 256, 0, st>>>(static_cast<float *>(D[0]),
                                                static_cast<float *>(M[0]), dJdc, n,
                                                (size_t)nx);
  HIPCHK(h, hipGetLastError());
  int cur = 0;
  const int64_t N = h->rec_steps, K = h->rec_K;
  const int64_t nseg = (N + K - 1) / K;
  if (nseg > A.nchk || K > A.K) return fail(h, LBE_CSF_EINVAL, "record exceeds the workspace");
  const bool vartau = h->base.dtauf != 0.0 || h->base.dtauT != 0.0;
  AdjArgs aa;
  aa.s = h->base;
  aa.a = Abuf;
  aa.part = part;
  aa.dtw = tw;
  aa.ntx = ntx;
  char *chk0 = base + A.off_chk;
  // Tapes.  With c-dependent relaxation times the first tape holds all K
  // states of a segment and its K moment sets.  With constant ones a segment
  // needs two rotating state slots and its moment sets, and two tapes
  // alternate: the replay of segment k - 1 fills one on a second stream while
  // the adjoint steps of segment k read the other (events order the reuse).
  char *tape_base[2] = {base + A.off_tape, base + A.off_tape2};
  const size_t tape_states[2] = {(size_t)A.K, 2};
  const bool overlap = !vartau && nseg > 1;
  hipEvent_t ev_start = nullptr, ev_rep[2] = {nullptr, nullptr}, ev_adj[2] = {nullptr, nullptr};
  // the events are released on every way out of this function
  struct EventSet {
    hipEvent_t *e[5];
    ~EventSet() {
      for (hipEvent_t *p : e)
        if (*p) (void)hipEventDestroy(*p);
    }
  } event_set{{&ev_start, &ev_rep[0], &ev_rep[1], &ev_adj[0], &ev_adj[1]}};
  if (overlap) {
    bool ok = true;
    if (!h->aux) {
      // on the handle's device, at the default priority
      int prev = 0;
      ok = hipGetDevice(&prev) == hipSuccess;
      if (ok && prev != h->device) ok = hipSetDevice(h->device) == hipSuccess;
      ok = ok && hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) == hipSuccess;
      if (prev != h->device) (void)hipSetDevice(prev);
    }
    for (hipEvent_t *e : {&ev_start, &ev_rep[0], &ev_rep[1], &ev_adj[0], &ev_adj[1]})
      ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
    // the replays on the second stream start after everything queued so far
    ok = ok && hipEventRecord(ev_start, st) == hipSuccess;
    if (!ok) return fail(h, LBE_CSF_EDEVICE, "backward: could not set up the second stream");
  }
  auto seg_len = [&](int64_t k) { return std::min(K, N - k * K); };
  // state j of segment k on tape b: the checkpoint, then the tape slots
  auto state = [&](int64_t k, int b, int64_t j) -> void * {
    if (j == 0) return chk0 + (size_t)k * A.state_bytes;
    return tape_base[b] + (size_t)(vartau ? j : (j & 1)) * A.state_bytes;
  };
  auto moments = [&](int b, int64_t j) -> void * {
    return tape_base[b] + tape_states[b] * A.state_bytes + (size_t)j * A.mom_bytes;
  };
  // the forward steps of segment k from its checkpoint, writing the moment
  // tape (and, with c-dependent relaxation times, keeping the states)
  auto replay = [&](int64_t k, int b, hipStream_t on) {
    const int64_t m = seg_len(k);
    for (int64_t j = 0; j < m; ++j) {
      const bool last = j + 1 == m;   // its successor is not needed
      const int rc = launch_step_on(h, on, last ? kTape : (kStore | kTape), state(k, b, j),
                                    last ? nullptr : state(k, b, j + 1), nullptr, nullptr,
                                    nullptr, nullptr, nullptr, moments(b, j));
      if (rc != LBE_CSF_OK) return rc;
    }
    return (int)LBE_CSF_OK;
  };
  auto tape_of = [&](int64_t k) { return overlap ? (int)(k & 1) : 0; };
  if (overlap) {
    const int rc = replay(nseg - 1, tape_of(nseg - 1), st);
    if (rc != LBE_CSF_OK) return rc;
  }
  for (int64_t k = nseg - 1; k >= 0; --k) {
    const int64_t m = seg_len(k);
    const int b = tape_of(k);
    if (overlap) {
      if (k > 0) {
        // segment k - 1 into the other tape, once the adjoint steps of
        // segment k + 1 (which read that tape) are done
        const int bn = tape_of(k - 1);
        hipError_t e = hipStreamWaitEvent(h->aux, k + 1 < nseg ? ev_adj[bn] : ev_start, 0);
        int rc = e == hipSuccess ? replay(k - 1, bn, h->aux) : (int)LBE_CSF_EDEVICE;
        if (rc == LBE_CSF_OK && hipEventRecord(ev_rep[bn], h->aux) != hipSuccess)
          rc = LBE_CSF_EDEVICE;
        if (rc != LBE_CSF_OK)
          return rc == LBE_CSF_EDEVICE ? fail(h, rc, "backward: second stream") : rc;
      }
      if (k < nseg - 1 && hipStreamWaitEvent(st, ev_rep[b], 0) != hipSuccess)
        return fail(h, LBE_CSF_EDEVICE, "backward: stream wait");
    } else {
      const int rc = replay(k, b, st);
      if (rc != LBE_CSF_OK) return rc;
    }
    for (int64_t j = m - 1; j >= 0; --j) {
      aa.s.src = vartau ? state(k, b, j) : nullptr;
      aa.s.tape = moments(b, j);
      aa.d_in = D[cur];
      aa.m_in = M[cur];
      aa.d_out = D[1 - cur];
      aa.m_out = M[1 - cur];
      const bool curv = h->P.csf_form == 1;
      if (f64) {
        if (curv) launch_adj<double, false, true>(vartau, aa, nb, st);
        else launch_adj<double, false, false>(vartau, aa, nb, st);
      } else {
        if (curv) launch_adj<float, true, true>(vartau, aa, nb, st);
        else launch_adj<float, true, false>(vartau, aa, nb, st);
      }
      if (hipGetLastError() != hipSuccess)
        return fail(h, LBE_CSF_EDEVICE, "backward: adjoint kernel launch");
      cur = 1 - cur;
    }
    if (overlap && hipEventRecord(ev_adj[b], st) != hipSuccess) {
      return fail(h, LBE_CSF_EDEVICE, "backward: event record");
    }
  }
  const unsigned g1 = (unsigned)((n + 255) / 256);
  if (dF0 || dT0) {
    if (f64)
      adj_finish_kernel<double><<<g1, 256, 0, st>>>(static_cast<const double *>(D[cur]),
                                                    static_cast<const double *>(M[cur]), dF0,
                                                    dT0, n, (size_t)nx, h->base.rcv);
    else
      adj_finish_kernel<float><<<g1, 256, 0, st>>>(static_cast<const float *>(D[cur]),
                                                   static_cast<const float *>(M[cur]), dF0,
                                                   dT0, n, (size_t)nx, h->base.rcv);
  }
  adj_sum_kernel<<<1, 256, 0, st>>>(part, nb, outv);
  HIPCHK(h, hipGetLastError());
  if (dTw) HIPCHK(h, hipMemcpyAsync(dTw, tw, 2 * (size_t)nx * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(h, hipMemcpyAsync(dsT, outv, sizeof(double), hipMemcpyDeviceToHost, st));
  // the stream has waited for every replay of the second stream
  HIPCHK(h, hipStreamSynchronize(st));
  return LBE_CSF_OK;
}

void to_public(const DiagRecord &r, lbe_csf_diag *o) {
  o->step = r.step;
  o->mass = r.v[0];
  o->energy = r.v[1];
  o->sum_cy = r.v[2];
  o->sum_cx = r.v[3];
  o->mass_thr = r.v[4];
  o->sum_cuy_thr = r.v[5];
  o->centroid_y = r.v[0] != 0.0 ? r.v[2] / r.v[0] : NAN;
  o->u_r = r.v[4] != 0.0 ? r.v[5] / r.v[4] : NAN;
  o->n_nonfinite = (int64_t)r.v[6];
}

// Scratch of lbe_csf_diagnostics_noalloc: the per-block partial sums of one
// diagnostic launch, then one record.  A file-scope device array, so that the
// call needs no device memory from the caller or the runtime; every GPU the
// library runs on holds its own copy until the process ends.  Host code uses
// only the address that hipGetSymbolAddress returns for the current device
// (the array's name is not a device address on the host).
constexpr int kScratchMaxBlocks = 16384;
constexpr size_t kScratchDoubles =
    (size_t)kScratchMaxBlocks * kNumPartials + (sizeof(DiagRecord) + 7) / 8;
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch array (looked up once per device, with
// that device current); nullptr and a message on failure.
double *scratch_on(int device, std::string *why) {
  if (device < 0 || device >= kMaxDevices) {
    *why = "device ordinal out of range";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      *why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_ptr[device] = static_cast<double *>(ptr);
  }
  return g_scratch_ptr[device];
}

}  // namespace

extern "C" {

int lbe_csf_workspace_size(const lbe_csf_params *params, int64_t record_steps,
                           size_t *bytes) {
  std::string why;
  if (!params_valid(params, &why)) return fail(nullptr, LBE_CSF_EINVAL, why);
  if (!bytes) return fail(nullptr, LBE_CSF_EINVAL, "bytes is NULL");
  if (record_steps < 0) return fail(nullptr, LBE_CSF_EINVAL, "record_steps < 0");
  *bytes = make_layout(params, record_steps).total;
  return LBE_CSF_OK;
}

int lbe_csf_create(const lbe_csf_params *params, void *workspace, size_t bytes,
                   int64_t record_steps, void *stream, const double *phi0,
                   const double *T0, const double *Twall_bot,
                   const double *Twall_top, lbe_csf **out) {
  std::string why;
  if (!out) return fail(nullptr, LBE_CSF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!params_valid(params, &why)) return fail(nullptr, LBE_CSF_EINVAL, why);
  if (!workspace || !phi0 || !T0) return fail(nullptr, LBE_CSF_EINVAL, "NULL device pointer");
  if (params->walls_y && (!Twall_bot || !Twall_top))
    return fail(nullptr, LBE_CSF_EINVAL, "wall temperatures required with walls_y = 1");
  if (record_steps < 0) return fail(nullptr, LBE_CSF_EINVAL, "record_steps < 0");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(nullptr, LBE_CSF_EINVAL, "workspace not 256-byte aligned");
  const Layout L = make_layout(params, record_steps);
  if (bytes < L.total)
    return fail(nullptr, LBE_CSF_ENOMEM,
                "workspace too small: need " + std::to_string(L.total) + " bytes");
  lbe_csf *h = new (std::nothrow) lbe_csf();
  if (!h) return fail(nullptr, LBE_CSF_ENOMEM, "host allocation failed");
  h->P = *params;
  h->L = L;
  h->la = launch_for(params, L.state_bytes);
  h->small_lds = 0;
  h->small_res = false;
  h->tile = use_tile_kernel(params);
  h->diag_blocks = h->tile ? tile_blocks(params->nx, params->ny) : h->la.nblocks;
  h->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
  {
    // small grids: many plain steps per launch when the moments of the
    // whole grid fit in one block's LDS
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) !=
        hipSuccess)
      max_lds = 0;
    // both states in LDS where they fit, else the moments only
    const bool f64 = params->precision == LBE_CSF_FP64;
    const size_t lds_res = small_res_bytes(params), lds = small_lds_bytes(params);
    if (lds_res > 0 && lds_res <= (size_t)max_lds) {
      const hipError_t e = f64 ? small_attrs<double, double, false, true>(lds_res)
                               : small_attrs<float, float, true, true>(lds_res);
      if (e == hipSuccess) {
        h->small_lds = lds_res;
        h->small_res = true;
      }
      (void)hipGetLastError();
    }
    if (h->small_lds == 0 && lds > 0 && lds <= (size_t)max_lds) {
      const hipError_t e = f64 ? small_attrs<double, double, false, false>(lds)
                               : small_attrs<float, float, true, false>(lds);
      if (e == hipSuccess) h->small_lds = lds;
      (void)hipGetLastError();
    }
  }
  h->ws = static_cast<char *>(workspace);
  h->state[0] = h->ws + L.off_a;
  h->state[1] = h->ws + L.off_b;
  h->cur = 0;
  h->step = 0;
  h->tw = reinterpret_cast<double *>(h->ws + L.off_tw);
  h->partials = reinterpret_cast<double *>(h->ws + L.off_part);
  h->ring = reinterpret_cast<DiagRecord *>(h->ws + L.off_ring);
  h->counters = reinterpret_cast<int64_t *>(h->ws + L.off_cnt);
  h->rec = reinterpret_cast<DiagRecord *>(h->ws + L.off_rec);
  h->record_cap = record_steps;
  h->recorded = false;
  fill_constants(h);
  const int nx = params->nx, ny = params->ny;
  auto cleanup = [&](int rc) {
    if (rc != LBE_CSF_OK) {
      g_create_error = h->err;
      delete h;
    }
    return rc;
  };
  hipError_t e = hipSuccess;
  if (params->walls_y) {
    e = hipMemcpyAsync(h->tw, Twall_bot, nx * sizeof(double), hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->tw + nx, Twall_top, nx * sizeof(double), hipMemcpyDeviceToDevice,
                         h->stream);
  } else {
    e = hipMemsetAsync(h->tw, 0, 2 * nx * sizeof(double), h->stream);
  }
  if (e == hipSuccess) e = hipMemsetAsync(h->counters, 0, 4 * sizeof(int64_t), h->stream);
  if (e != hipSuccess) {
    h->err = std::string("copy of wall temperatures: ") + hipGetErrorString(e);
    return cleanup(LBE_CSF_EDEVICE);
  }
  const double beta2 = h->base.beta2, eps2 = h->base.eps2, gam3 = h->base.gam3;
  dim3 grid((nx + 255) / 256, ny);
  if (params->precision == LBE_CSF_FP64)
    init_kernel<double, false><<<grid, 256, 0, h->stream>>>(
        static_cast<double *>(h->state[0]), phi0, T0, nx, ny, params->walls_y, beta2, eps2,
        gam3, h->base.rcv, params->p0, 0.0, 0.0, h->base.rho, h->base.drho, h->base.cv);
  else
    init_kernel<float, true><<<grid, 256, 0, h->stream>>>(
        static_cast<float *>(h->state[0]), phi0, T0, nx, ny, params->walls_y, beta2, eps2,
        gam3, h->base.rcv, params->p0, params->T_shift, params->T_grad, h->base.rho,
        h->base.drho, h->base.cv);
  e = hipGetLastError();
  if (e != hipSuccess) {
    h->err = std::string("init kernel: ") + hipGetErrorString(e);
    return cleanup(LBE_CSF_EDEVICE);
  }
  *out = h;
  return LBE_CSF_OK;
}

int lbe_csf_step(lbe_csf *h, int64_t nsteps, int32_t record) {
  if (!h) return LBE_CSF_EINVAL;
  if (nsteps < 0) return fail(h, LBE_CSF_EINVAL, "nsteps < 0");
  if (record && h->base.drho != 0.0)
    return fail(h, LBE_CSF_EINVAL, "the adjoint covers one density only");
  if (record && (nsteps == 0 || nsteps > h->record_cap))
    return fail(h, LBE_CSF_EINVAL,
                "record needs 0 < nsteps <= record_steps of the workspace (" +
                    std::to_string(h->record_cap) + ")");
  h->recorded = false;
  int64_t K = 0;
  if (record) {
    K = adj_segment_length(nsteps);
    h->rec_start = h->step;
    h->rec_steps = nsteps;
    h->rec_K = K;
  }
  const int de = h->P.diag_every;
  bool any_diag = false;
  for (int64_t s = 0; s < nsteps; ++s) {
    if (!record && h->small_lds > 0) {
      // the plain steps up to the next diagnostic step, many per launch
      int64_t run = nsteps - s;
      if (de > 0) run = std::min<int64_t>(run, (de - h->step % de) % de);
      if (run > 0) {
        const int rc = launch_small(h, run);
        if (rc != LBE_CSF_OK) return rc;
        s += run - 1;
        continue;
      }
    }
    if (record && s % K == 0) {
      // checkpoint F_{start + s}
      const int rc = adj_save_checkpoint(h->ws + h->L.off_adj, h->L.adj, s / K,
                                         h->state[h->cur], h->L.state_bytes, h->stream);
      if (rc != 0) return fail(h, LBE_CSF_EDEVICE, "checkpoint copy failed");
    }
    const bool diag = de > 0 && (h->step % de == 0);
    int rc = launch_step(h, diag ? (kStore | kDiag) : kStore, h->state[h->cur],
                         h->state[1 - h->cur], nullptr, nullptr, nullptr, nullptr, nullptr);
    if (rc != LBE_CSF_OK) return rc;
    if (diag) {
      rc = launch_reduce(h, h->step, true);
      if (rc != LBE_CSF_OK) return rc;
      any_diag = true;
    }
    h->cur = 1 - h->cur;
    h->step += 1;
  }
  if (record) h->recorded = true;
  if (any_diag) {
    int64_t cnt[2];
    HIPCHK(h, hipMemcpyAsync(cnt, h->counters, sizeof(cnt), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (cnt[1] > 0) {
      return fail(h, LBE_CSF_ENONFINITE,
                  std::to_string(cnt[1]) + " non-finite site values in diagnostics");
    }
  }
  return LBE_CSF_OK;
}

int lbe_csf_fields(lbe_csf *h, double *phi, double *ux, double *uy, double *p, double *T) {
  if (!h) return LBE_CSF_EINVAL;
  return launch_step(h, kFields, h->state[h->cur], nullptr, phi, ux, uy, p, T);
}

int lbe_csf_diagnostics(lbe_csf *h, lbe_csf_diag *out) {
  if (!h || !out) return h ? fail(h, LBE_CSF_EINVAL, "out is NULL") : LBE_CSF_EINVAL;
  int rc = launch_step(h, kDiag, h->state[h->cur], nullptr, nullptr, nullptr, nullptr,
                       nullptr, nullptr);
  if (rc != LBE_CSF_OK) return rc;
  rc = launch_reduce(h, h->step, false);
  if (rc != LBE_CSF_OK) return rc;
  DiagRecord r;
  HIPCHK(h, hipMemcpyAsync(&r, h->rec, sizeof(r), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  to_public(r, out);
  return LBE_CSF_OK;
}

int lbe_csf_diagnostics_noalloc(lbe_csf *h, lbe_csf_diag *out) {
  if (!h || !out) return h ? fail(h, LBE_CSF_EINVAL, "out is NULL") : LBE_CSF_EINVAL;
  if (h->diag_blocks > kScratchMaxBlocks)
    return fail(h, LBE_CSF_EINVAL,
                "diagnostics_noalloc: the launch has " + std::to_string(h->diag_blocks) +
                    " blocks, the static scratch holds the partials of at most " +
                    std::to_string(kScratchMaxBlocks));
  int prev = 0;
  HIPCHK(h, hipGetDevice(&prev));
  if (prev != h->device) HIPCHK(h, hipSetDevice(h->device));
  std::string why;
  double *ptr = scratch_on(h->device, &why);
  int rc = LBE_CSF_OK;
  if (!ptr) {
    rc = fail(h, LBE_CSF_EDEVICE, why);
  } else {
    // every block writes its own partials and the reduction writes the
    // record, so nothing needs clearing first
    double *partials = ptr;
    DiagRecord *rec = reinterpret_cast<DiagRecord *>(ptr + (size_t)kScratchMaxBlocks * kNumPartials);
    rc = launch_step(h, kDiag, h->state[h->cur], nullptr, nullptr, nullptr, nullptr, nullptr,
                     nullptr, nullptr, partials);
    if (rc == LBE_CSF_OK) {
      diag_reduce_kernel<<<1, 256, 0, h->stream>>>(partials, h->diag_blocks, rec, 1, nullptr,
                                                   h->step);
      DiagRecord r;
      hipError_t e = hipGetLastError();
      if (e == hipSuccess)
        e = hipMemcpyAsync(&r, rec, sizeof(r), hipMemcpyDeviceToHost, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      if (e != hipSuccess)
        rc = fail(h, LBE_CSF_EDEVICE, std::string("diagnostics_noalloc: ") + hipGetErrorString(e));
      else
        to_public(r, out);
    }
  }
  if (prev != h->device) (void)hipSetDevice(prev);
  return rc;
}

int lbe_csf_diag_history(lbe_csf *h, lbe_csf_diag *out, int32_t max, int32_t *count) {
  if (!h) return LBE_CSF_EINVAL;
  if (!count || (max > 0 && !out)) return fail(h, LBE_CSF_EINVAL, "NULL output");
  int64_t cnt[2];
  HIPCHK(h, hipMemcpyAsync(cnt, h->counters, sizeof(cnt), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  const int64_t have = std::min<int64_t>(cnt[0], kDiagRing);
  const int64_t ncopy = std::min<int64_t>(have, std::max(0, max));
  const int64_t first = cnt[0] - have;
  if (ncopy > 0) {
    // the oldest ncopy records: one contiguous range of the ring, or two
    // when it wraps
    std::vector<DiagRecord> buf((size_t)ncopy);
    const int64_t start = first % kDiagRing;
    const int64_t part1 = std::min<int64_t>(ncopy, kDiagRing - start);
    HIPCHK(h, hipMemcpyAsync(buf.data(), h->ring + start, (size_t)part1 * sizeof(DiagRecord),
                             hipMemcpyDeviceToHost, h->stream));
    if (part1 < ncopy)
      HIPCHK(h, hipMemcpyAsync(buf.data() + part1, h->ring,
                               (size_t)(ncopy - part1) * sizeof(DiagRecord),
                               hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int64_t k = 0; k < ncopy; ++k) to_public(buf[(size_t)k], &out[k]);
  }
  *count = (int32_t)ncopy;
  int64_t zero[2] = {0, cnt[1]};
  HIPCHK(h, hipMemcpyAsync(h->counters, zero, sizeof(zero), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return LBE_CSF_OK;
}

int lbe_csf_get_state(lbe_csf *h, double *F) {
  if (!h) return LBE_CSF_EINVAL;
  if (!F) return fail(h, LBE_CSF_EINVAL, "F is NULL");
  const size_t n = (size_t)h->P.nx * h->P.ny;
  dim3 grid((unsigned)((n + 255) / 256), 27);
  if (h->P.precision == LBE_CSF_FP64)
    state_to_f64<double, false><<<grid, 256, 0, h->stream>>>(
        static_cast<const double *>(h->state[h->cur]), F, h->P.nx, h->P.ny, 0.0, 0.0, 0.0, 0.0);
  else
    state_to_f64<float, true><<<grid, 256, 0, h->stream>>>(
        static_cast<const float *>(h->state[h->cur]), F, h->P.nx, h->P.ny, h->base.p0,
        h->base.rcv, h->base.Ts, h->base.Tg);
  HIPCHK(h, hipGetLastError());
  return LBE_CSF_OK;
}

int lbe_csf_set_state(lbe_csf *h, const double *F) {
  if (!h) return LBE_CSF_EINVAL;
  if (!F) return fail(h, LBE_CSF_EINVAL, "F is NULL");
  const size_t n = (size_t)h->P.nx * h->P.ny;
  dim3 grid((unsigned)((n + 255) / 256), 27);
  if (h->P.precision == LBE_CSF_FP64)
    state_from_f64<double, false><<<grid, 256, 0, h->stream>>>(
        static_cast<double *>(h->state[h->cur]), F, h->P.nx, h->P.ny, 0.0, 0.0, 0.0, 0.0);
  else
    state_from_f64<float, true><<<grid, 256, 0, h->stream>>>(
        static_cast<float *>(h->state[h->cur]), F, h->P.nx, h->P.ny, h->base.p0,
        h->base.rcv, h->base.Ts, h->base.Tg);
  HIPCHK(h, hipGetLastError());
  h->recorded = false;
  return LBE_CSF_OK;
}

int64_t lbe_csf_step_count(const lbe_csf *h) { return h ? h->step : -1; }

int lbe_csf_backward(lbe_csf *h, const double *dJ_dc, double *dJ_dsigmaT, double *dJ_dTwall,
                     double *dJ_dF0, double *dJ_dT0) {
  if (!h) return LBE_CSF_EINVAL;
  if (!h->recorded || h->step != h->rec_start + h->rec_steps)
    return fail(h, LBE_CSF_ENOTRECORDED, "no recorded run ends at the current state");
  if (!dJ_dc || !dJ_dsigmaT) return fail(h, LBE_CSF_EINVAL, "NULL seed or output");
  return run_backward(h, dJ_dc, dJ_dsigmaT, dJ_dTwall, dJ_dF0, dJ_dT0);
}

void lbe_csf_destroy(lbe_csf *h) { delete h; }

const char *lbe_csf_strerror(int status) {
  switch (status) {
    case LBE_CSF_OK: return "ok";
    case LBE_CSF_EINVAL: return "invalid argument";
    case LBE_CSF_ENOMEM: return "workspace too small";
    case LBE_CSF_EDEVICE: return "device error";
    case LBE_CSF_ENOTRECORDED: return "no recorded forward run";
    case LBE_CSF_ENONFINITE: return "non-finite values in the state";
    default: return "unknown status";
  }
}

const char *lbe_csf_last_error(const lbe_csf *h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
