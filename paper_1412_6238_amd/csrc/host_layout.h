// host_layout.h -- host-side logic of liblbe_csf without HIP: the sizes of a
// state, the caller's workspace layout, the launch shape of the step kernel
// and the parameter checks.  The library includes it; so does a CPU test
// driver built with address and undefined-behaviour sanitizers.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>

#include "../../include/lbe_csf.h"

namespace lbe {

constexpr int kNumS = 25;  // planes in the storage type; the two rest planes follow

// Storage of the two rest populations (g_0, then hbar_0) after the 25 planes.
// The FP64 form keeps both in FP64.  The FP32 form keeps g_0 in FP64 and
// hbar_0 in FP32: c sits almost entirely in g_0, and its rounding enters the
// force through eps^2 lap c (stored in FP32, or as 30-bit fixed point, g_0
// gave the planar Marangoni velocity errors of 14% and 0.4% against the FP64
// path), while hbar_0 is stored as the deviation from w_0 rho cv Tr(y), which
// FP32 holds to far below the thermal signal (largest error 6e-6 in T over
// the test cases).
enum : int { kRestF64 = 0, kRestF32 = 1 };
template <typename S>
constexpr int rest_fmt(int which) {
  return sizeof(S) == 8 || which == 0 ? kRestF64 : kRestF32;
}
template <typename S>
constexpr uint32_t rest_bytes(int which) {
  return rest_fmt<S>(which) == kRestF64 ? 8u : 4u;
}
// bytes of one state of n sites
template <typename S>
constexpr size_t state_bytes_for(size_t n) {
  return kNumS * n * sizeof(S) + n * (rest_bytes<S>(0) + rest_bytes<S>(1));
}
// The state is row-interleaved: row y is one record of row_bytes<S>(nx)
// bytes that holds the row's nx values of each of the 25 storage planes in
// turn (plane p at p * nx * sizeof(S)), then those of g_0 and of hbar_0 (at
// rest_base<S>(0 or 1, nx)).  A row's 27 segments are thus contiguous, which
// a row-marching step reads and writes as one stream per row instead of 27
// streams a plane apart.
template <typename S>
constexpr size_t row_bytes(size_t nx) {
  return state_bytes_for<S>(nx);
}
template <typename S>
constexpr size_t rest_base(int which, size_t nx) {
  return kNumS * nx * sizeof(S) + (which ? nx * rest_bytes<S>(0) : 0);
}

// small-grid kernel: LDS bytes of the moments c (FP64), T and p (R) of the
// grid with a halo column on each side and a row beyond each y boundary,
// rounded up to 16 bytes (the resident states follow)
template <typename R>
constexpr size_t small_moment_bytes(size_t nx, size_t ny) {
  return ((nx + 2) * (ny + 2) * (8 + 2 * sizeof(R)) + 15) / 16 * 16;
}
// ... which takes grids of up to this many sites, one per lane of a block
// of at most as many lanes
constexpr int kSmallMaxSites = 512;
// tile kernel (latency-bound grids): tiles of kTileX x kTileY sites, one per
// lane of a block
constexpr int kTileX = 64, kTileY = 4;
inline int tile_blocks(int nx, int ny) {
  return ((nx + kTileX - 1) / kTileX) * ((ny + kTileY - 1) / kTileY);
}

constexpr int kNumPartials = 7;  // mass, energy, cy, cx, mass_thr, cuy_thr, nonfinite

// one diagnostic record: the step and the seven FP64 sums
struct DiagRecord {
  int64_t step;
  double v[kNumPartials];
};

constexpr int kAdjTX = 64;   // adjoint tile: 64 columns x 4 rows, one site per thread
constexpr int kAdjTY = 4;
// stencil cotangent planes: grad c, lap c, grad T, grad p, and the Hessian of
// c (hxx, hxy, hyy; read by the curvature form only)
constexpr int kAdjA = 10;

struct AdjLayout {
  int64_t record_steps;   // capacity N
  int64_t K;              // checkpoint spacing for N steps
  int64_t nchk;           // checkpoints ceil(N / K)
  size_t state_bytes;     // one state (aligned)
  size_t mom_bytes;       // one moment set: c (FP64), T, p, jx, jy
  size_t plane_bytes;     // one plane of the arithmetic type
  size_t off_chk;         // nchk states
  size_t off_tape;        // K states, then K moment sets
  size_t off_tape2;       // a second tape, 2 states and K moment sets: with
                          // constant relaxation times the replay of the next
                          // segment fills it while the adjoint steps read the first
  size_t off_lam;         // D x2 (27 planes), M x2 (3 planes), A (kAdjA planes)
  size_t off_part;        // per-block FP64 partial sums of dJ/dsigmaT
  size_t off_tw;          // FP64 [2][nx] dJ/dTwall accumulators
  size_t off_out;         // FP64 scalar result
  size_t total;
};

inline int64_t adj_segment_length(int64_t nsteps) {
  if (nsteps <= 1) return 1;
  int64_t K = (int64_t)std::ceil(std::sqrt((double)nsteps));
  while (K * K < nsteps) ++K;
  while (K > 1 && (K - 1) * (K - 1) >= nsteps) --K;
  return K;
}

inline int adj_tiles_x(int nx) { return (nx + kAdjTX - 1) / kAdjTX; }
inline int adj_tiles_y(int ny) { return (ny + kAdjTY - 1) / kAdjTY; }

inline AdjLayout adj_layout(int nx, int ny, size_t state_bytes, size_t value_bytes,
                            int64_t record_steps) {
  AdjLayout A{};
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  A.record_steps = record_steps;
  if (record_steps <= 0) return A;
  const size_t n = (size_t)nx * ny;
  A.state_bytes = al(state_bytes);
  A.mom_bytes = al(n * (8 + 4 * value_bytes));
  A.plane_bytes = al(n * value_bytes);
  A.K = adj_segment_length(record_steps);
  A.nchk = (record_steps + A.K - 1) / A.K;
  size_t o = 0;
  A.off_chk = o; o += (size_t)A.nchk * A.state_bytes;
  A.off_tape = o; o += (size_t)A.K * (A.state_bytes + A.mom_bytes);
  A.off_tape2 = o; o += 2 * A.state_bytes + (size_t)A.K * A.mom_bytes;
  A.off_lam = o; o += (2 * 27 + 2 * 3 + kAdjA) * A.plane_bytes;
  A.off_part = o; o += al((size_t)adj_tiles_x(nx) * adj_tiles_y(ny) * sizeof(double));
  A.off_tw = o; o += al(2 * (size_t)nx * sizeof(double));
  A.off_out = o; o += 256;
  A.total = o;
  return A;
}

namespace host {

constexpr int kDiagRing = 4096;
constexpr int kNumCUs = 256;   // compute units of an MI355X (gfx950)
constexpr size_t kLastLevelCache = size_t(256) << 20;   // MI355X Infinity Cache
constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Launch {
  int pipe;      // row pipeline of the step kernel (see step_kernel.h)
  int nw;        // waves per block (strip width 64 * nw)
  int nstrips;
  int rows;      // rows per chunk
  int nchunks;
  int nblocks;
  bool stream;   // plain FP32 steps use kStream (state beyond the last-level cache)
};

// two_ahead: the step may load rows two ahead (not with two densities, whose
// step loads one row ahead)
inline Launch pick_launch(int nx, int ny, bool fp32, bool two_ahead) {
  Launch L;
  // Strip width: FP32 four waves on wide grids, two from 256 columns; a
  // narrower grid takes one strip across its whole width with at least two
  // waves (measured 6-20% faster than one-wave strips on 8- to 200-column
  // grids).  FP64 four waves at every width: on the row-interleaved state,
  // on eleven grids below one block per CU, 1.5-13% faster than two waves on
  // seven (256 x 512: 17.2 against 19.4 us; 1024 x 64: 11.0 against 12.6)
  // and within 1% on the other four.
  L.nw = !fp32 ? 4 : (nx >= 2048 ? 4 : (nx >= 256 ? 2 : (nx > 128 ? 4 : 2)));
  if (const char *e = std::getenv("LBE_CSF_NW")) {
    const int v = std::atoi(e);
    if (v == 1 || v == 2 || v == 4 || v == 8) L.nw = v;
  }
  const int bx = 64 * L.nw;
  L.nstrips = (nx + bx - 1) / bx;
  // Row chunks: about 2048 waves (two per SIMD) resident at once -- long
  // chunks on large grids (fewer halo rows re-read), down to one row per
  // block on small grids, where parallelism is the limit.  The FP32 step on a
  // large grid loads rows two ahead (PIPE 2, which needs the registers of a
  // two-wave occupancy) and runs best with twice as many, shorter chunks.
  auto rows_for = [&](long long waves) {
    const long long want = std::max(1LL, waves / ((long long)L.nw * L.nstrips));
    return (int)std::max<long long>(1, (ny + want - 1) / want);
  };
  int rows = rows_for(2048);
  L.pipe = 1;
  // One block per CU marching long chunks: eight-wave strips loading rows
  // two ahead in the FP32 step, four-wave strips loading one row ahead in
  // FP64.  Measured on the row-interleaved state against the shapes below
  // (interleaved timing windows after a warm-up, nine grids from 1024 x 512
  // to 8192 x 1024): FP32 up to 11% faster and none slower (the same on
  // 4096^2 and 8192 x 1024, which already had this shape), FP64 2-8% faster
  // everywhere, and within 1.5% of the best shape of a wider sweep.  With two
  // densities FP64 gains 0.3-6% on four grids; the FP32 form (rows one ahead)
  // keeps the shapes below, which were as fast or within 4%.  Taken when the
  // chunks are at least four rows long.
  const int nw1 = fp32 ? 8 : 4;
  const int nstr1 = (nx + 64 * nw1 - 1) / (64 * nw1);
  const int chunks1 = std::max(1, kNumCUs / nstr1);
  const int rows1 = (ny + chunks1 - 1) / chunks1;
  const bool one_per_cu = (two_ahead || !fp32) && nx >= 64 * nw1 && rows1 >= 4;
  if (one_per_cu && !std::getenv("LBE_CSF_NW")) {
    L.nw = nw1;
    L.nstrips = nstr1;
    rows = rows1;
    L.pipe = fp32 ? 2 : 1;
  } else if (fp32 && rows >= 64) {
    rows = rows_for(4096);
    L.pipe = 2;
  } else if (fp32 && rows >= 4) {
    L.pipe = 2;
  } else if (!fp32 && rows >= 64) {
    rows = rows_for(3072);   // measured on 4096^2: 86-row chunks beat 64 and 128
  }
  if (const char *e = std::getenv("LBE_CSF_PIPE")) {
    const int v = std::atoi(e);
    if (v == 0 || v == 1 || v == 2) L.pipe = v;
  }
  // two densities load rows one ahead; their FP32 form keeps the shapes
  // after the one-block-per-CU rule: 4-wave strips with 64-row chunks on
  // 4096^2 (measured 11.9k MLUPS, against 10.7k on eight-wave strips, on the
  // earlier plane-by-plane state)
  if (!two_ahead) L.pipe = 1;
  if (const char *e = std::getenv("LBE_CSF_ROWS")) {
    const int v = std::atoi(e);
    if (v >= 1) rows = v;
  }
  L.rows = std::min(rows, ny);
  L.nchunks = (ny + L.rows - 1) / L.rows;
  L.nblocks = L.nstrips * L.nchunks;
  L.stream = false;
  return L;
}

// two fluid densities (rho2 > 0 and different from rho)
inline bool two_densities(const lbe_csf_params *p) { return p->rho2 > 0.0 && p->rho2 != p->rho; }

struct Layout {
  size_t state_bytes;
  size_t off_a, off_b, off_tw, off_part, off_ring, off_cnt, off_rec, off_pc, off_adj, total;
  AdjLayout adj;
};

inline bool params_valid(const lbe_csf_params *p, std::string *why) {
  auto bad = [&](const char *m) {
    if (why) *why = m;
    return false;
  };
  if (!p) return bad("params is NULL");
  if (p->nx < 3 || p->ny < 3) return bad("nx and ny must be >= 3");
  // the kernels address a state through one buffer descriptor (32-bit byte
  // offsets): 25 planes of the storage type plus two FP64 planes < 4 GiB
  const double sb = p->precision == LBE_CSF_FP64 ? (double)state_bytes_for<double>(1)
                                                 : (double)state_bytes_for<float>(1);
  if ((double)p->nx * (double)p->ny * sb >= 4294967296.0)
    return bad("grid too large: a state must stay below 4 GiB");
  if (p->walls_y != 0 && p->walls_y != 1) return bad("walls_y must be 0 or 1");
  if (p->precision != LBE_CSF_FP64 && p->precision != LBE_CSF_FP32_DEV)
    return bad("unknown precision");
  auto fin = [](double v) { return std::isfinite(v); };
  if (!(p->rho > 0) || !(p->cv > 0) || !fin(p->rho) || !fin(p->cv)) return bad("rho and cv must be > 0");
  for (int k = 0; k < 2; ++k) {
    if (!(p->tau_f[k] > 0.5) || !fin(p->tau_f[k])) return bad("tau_f must be > 1/2");
    if (!(p->tau_T[k] > 0.5) || !fin(p->tau_T[k])) return bad("tau_T must be > 1/2");
  }
  if (!(p->tau_g > 0.5) || !fin(p->tau_g)) return bad("tau_g must be > 1/2");
  if (!(p->mobility > 0) || !fin(p->mobility)) return bad("mobility must be > 0");
  if (!(p->width > 0) || !fin(p->width)) return bad("width must be > 0");
  if (!(p->beta > 0) || !fin(p->beta)) return bad("beta must be > 0");
  if (!fin(p->sigma0) || !fin(p->sigmaT) || !fin(p->Tref) || !fin(p->force[0]) ||
      !fin(p->force[1]) || !fin(p->p0) || !fin(p->T_shift) || !fin(p->T_grad))
    return bad("non-finite parameter");
  if (p->diag_every < 0) return bad("diag_every must be >= 0");
  if (p->csf_form != 0 && p->csf_form != 1) return bad("csf_form must be 0 or 1");
  if (!(p->rho2 >= 0.0) || !fin(p->rho2)) return bad("rho2 must be >= 0 (0: one density)");
  // the FP32 form's linear thermal reference T_shift + T_grad y is not
  // periodic: a population crossing a periodic y boundary would change
  // reference by T_grad ny instead of T_grad
  if (p->precision == LBE_CSF_FP32_DEV && p->walls_y == 0 && p->T_grad != 0.0)
    return bad("T_grad must be 0 with periodic y in the FP32 form");
  return true;
}

inline Layout make_layout(const lbe_csf_params *p, int64_t record_steps) {
  Layout L{};
  const size_t n = (size_t)p->nx * p->ny;
  const size_t vb = p->precision == LBE_CSF_FP64 ? 8 : 4;
  L.state_bytes = vb == 8 ? state_bytes_for<double>(n) : state_bytes_for<float>(n);
  const Launch la = pick_launch(p->nx, p->ny, p->precision == LBE_CSF_FP32_DEV, !two_densities(p));
  size_t o = 0;
  L.off_a = o; o = align_up(o + L.state_bytes);
  L.off_b = o; o = align_up(o + L.state_bytes);
  L.off_tw = o; o = align_up(o + 2 * (size_t)p->nx * 8);
  // diagnostic partials: one per block of the row-marching or the tile kernel
  const size_t nparts = (size_t)std::max(la.nblocks, tile_blocks(p->nx, p->ny));
  L.off_part = o; o = align_up(o + nparts * kNumPartials * 8);
  L.off_ring = o; o = align_up(o + (size_t)kDiagRing * sizeof(DiagRecord));
  L.off_cnt = o; o = align_up(o + 4 * sizeof(int64_t));
  L.off_rec = o; o = align_up(o + sizeof(DiagRecord));
  L.off_pc = o; o = align_up(o + (two_densities(p) ? n * 8 : 0));   // pressure of Eq. 9
  L.off_adj = o;
  L.adj = adj_layout(p->nx, p->ny, L.state_bytes, vb, record_steps);
  o = align_up(o + L.adj.total);
  L.total = o;
  return L;
}

// The launch of a handle: pick_launch, and the store policy -- the FP32
// one-density step streams whole-line stores past the last-level cache when
// one step's source and destination states do not fit in it
// (LBE_CSF_STREAM=0/1 forces it off/on for that step).
inline Launch launch_for(const lbe_csf_params *p, size_t state_bytes) {
  const bool fp32 = p->precision == LBE_CSF_FP32_DEV;
  Launch la = pick_launch(p->nx, p->ny, fp32, !two_densities(p));
  la.stream = fp32 && !two_densities(p) && 2 * state_bytes > kLastLevelCache;
  if (const char *e = std::getenv("LBE_CSF_STREAM")) {
    const int v = std::atoi(e);
    if (v == 0 || v == 1) la.stream = v == 1 && fp32 && !two_densities(p);
  }
  return la;
}

// Small grids: LDS bytes of the moments c (FP64), T and p of the whole grid
// with a halo column on each side and a row beyond each y boundary, when
// plain steps run many per launch of one block (small_step_kernel); 0 when
// the grid is not small enough or has two densities.  LBE_CSF_SMALL=0 turns
// the path off.  The limit is one site per lane of a 512-lane block.
// Measured on MI355X with the row-interleaved state (one launch per step ->
// this path): 16 x 32 FP32 5.80 -> 4.99 us per step with the moments in LDS,
// 4.47 with the states too; 8 x 64 FP64 7.55 -> 6.65.  On 20 x 30 (600
// sites, 640 lanes) the moments-only kernel was slower than one launch per
// step (6.13 against 5.78 us), and on 40 x 100 (four sites per lane, plane
// layout) one block took 26 us against 5.7: its CU serialises the arithmetic
// that one launch per step spreads over a hundred blocks.
inline size_t small_lds_bytes(const lbe_csf_params *p) {
  if (const char *e = std::getenv("LBE_CSF_SMALL"))
    if (std::atoi(e) == 0) return 0;
  const size_t n = (size_t)p->nx * p->ny;
  if (two_densities(p) || n > (size_t)kSmallMaxSites) return 0;
  return p->precision == LBE_CSF_FP64 ? small_moment_bytes<double>(p->nx, p->ny)
                                      : small_moment_bytes<float>(p->nx, p->ny);
}
// Steps in tiles of one site per lane (tile_step_kernel) instead of
// row-marching chunks, on grids above the small-grid path and up to 1.5M
// sites, with one density or two (LBE_CSF_TILE=0/1 forces the choice).
// Measured on MI355X in interleaved windows against the row-marching
// kernel, one density: FP32 4-42% faster up to 1.44M sites (1024^2: 40.3
// against 50.3 us; 1500 x 700: 41.2 against 52.1), 7-13% slower from 1.5M
// up (2048 x 1024: 111 against 98 us; 4096^2: 918 against 690); FP64 6-49%
// faster up to 2^19 sites (160 x 300: 7.1 against 12.6 us; 512 x 1024: 36.0
// against 45.5) and 3-19% faster up to 1.44M where the width is not a
// multiple of the row kernel's 256-column strips (800^2: 63.3 against 78.4;
// 1030 x 1000: 101 against 114), 1-3% slower where it is (1024^2, 2048 x
// 512).  Two densities: 13-45% faster on six grids from 64 x 64 to 1024^2
// (160 x 300 FP64: 11.8 against 21.5 us).  On grids two or four tiles wide
// whose last tile holds 1 to 8 columns this relies on the tile kernel's
// lanes beyond the last column colliding their wrapped sites: left idle,
// they made 200 x 100 FP32 take 8.7 us in tiles against 7.2 on the
// row-marching kernel; now 5.8.
inline bool use_tile_kernel(const lbe_csf_params *p) {
  if (const char *e = std::getenv("LBE_CSF_TILE")) return std::atoi(e) == 1;
  const size_t n = (size_t)p->nx * p->ny;
  if (n <= (size_t)kSmallMaxSites) return false;
  if (p->precision == LBE_CSF_FP64)
    return n <= (size_t)1 << 19 || (n <= 1500000 && p->nx % 256 != 0);
  return n <= 1500000;
}

// LDS of the variant that also keeps both states in LDS (small_step_kernel
// with RES): the moments, then the two states; 0 where the small-grid path is
// off or LBE_CSF_SMALL=1 asks for the moments-only variant.  Whether it fits
// is the caller's test against the device's limit (160 KB on MI355X: every
// FP32 small grid, FP64 grids up to about 340 sites).
inline size_t small_res_bytes(const lbe_csf_params *p) {
  const size_t m = small_lds_bytes(p);
  if (m == 0) return 0;
  if (const char *e = std::getenv("LBE_CSF_SMALL"))
    if (std::atoi(e) == 1) return 0;
  const size_t n = (size_t)p->nx * p->ny;
  return m + 2 * (p->precision == LBE_CSF_FP64 ? state_bytes_for<double>(n)
                                                 : state_bytes_for<float>(n));
}

}  // namespace host
}  // namespace lbe
