// adjoint.h -- reverse-mode differentiation of the fused step: checkpoint
// layout, the adjoint step kernel and its helpers.
//
// One step is F_{n+1} = Stream(Collide(F_n)).  Collide at site x depends on
// F_n(x) and, through the nine-point stencils, on the moments (c, T, p) of the
// eight neighbours.  For a cotangent lambda_{n+1} of F_{n+1} the adjoint step
// returns lambda_n = (dF_{n+1}/dF_n)^T lambda_{n+1} in two stages per row:
//   A  lambda* = Stream^T lambda_{n+1}: a pull from x + xi_i; at a wall the
//      reflected population of the same site, with the sign flip of the
//      anti-bounce-back for hbar (whose wall term 2 w rho cv T_wall gives
//      dJ/dT_wall).  Then the transpose of the site's collision (site_adjoint):
//      the direct cotangent of the 27 populations of x, and the cotangents
//      a(x) of its seven stencil values (grad c, lap c, grad T, grad p), plus
//      the site's share of dJ/dsigmaT;
//   B  the stencil transposes: the moments of site y collect a(x) from every x
//      whose stencil reads y (in the wall rows the ghost row mirrors c and p
//      and holds 2 T_wall - T, so T collects with a minus sign and T_wall
//      twice), and the moment cotangents go to the populations they sum
//      (p = sum f, c = sum g, rho cv T = sum hbar).
// Stage A at the strip edges needs moments one column further out, so a block
// of 64*NW lanes produces 64*NW - 2 output columns; stage A runs one row ahead
// of stage B, and the direct cotangent of a row waits one row in registers.
//
// The run is differentiated by sqrt(N) checkpointing: the forward run saves
// every K-th state (K = ceil(sqrt N)); the backward pass replays each segment
// from its checkpoint into a tape of K states and sweeps it in reverse.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "step_kernel.h"

namespace lbe {

struct AdjLayout {
  int64_t record_steps;   // capacity N
  int64_t K;              // checkpoint spacing for N steps
  int64_t nchk;           // checkpoints ceil(N / K)
  size_t state_bytes;     // one state (aligned)
  size_t lam_bytes;       // one adjoint state: 27 planes of the arithmetic type
  size_t off_chk;         // nchk states
  size_t off_tape;        // K states (a replayed segment)
  size_t off_lam;         // two adjoint states
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

inline AdjLayout adj_layout(int nx, size_t state_bytes, size_t lam_bytes, int nblocks,
                            int64_t record_steps) {
  AdjLayout A{};
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  A.record_steps = record_steps;
  if (record_steps <= 0) return A;
  A.state_bytes = al(state_bytes);
  A.lam_bytes = al(lam_bytes);
  A.K = adj_segment_length(record_steps);
  A.nchk = (record_steps + A.K - 1) / A.K;
  size_t o = 0;
  A.off_chk = o; o += (size_t)A.nchk * A.state_bytes;
  A.off_tape = o; o += (size_t)A.K * A.state_bytes;
  A.off_lam = o; o += 2 * A.lam_bytes;
  A.off_part = o; o += al((size_t)nblocks * sizeof(double));
  A.off_tw = o; o += al(2 * (size_t)nx * sizeof(double));
  A.off_out = o; o += 256;
  A.total = o;
  return A;
}

inline int adj_save_checkpoint(char *adj_base, const AdjLayout &A, int64_t k,
                               const void *state, size_t bytes, hipStream_t st) {
  if (k < 0 || k >= A.nchk) return 1;
  char *dst = adj_base + A.off_chk + (size_t)k * A.state_bytes;
  return hipMemcpyAsync(dst, state, bytes, hipMemcpyDeviceToDevice, st) == hipSuccess ? 0 : 1;
}

struct AdjArgs {
  StepArgs s;               // constants, geometry (s.nstrips, s.rows_per_chunk of
                            // the adjoint launch) and F_n in s.src
  const void *lam_in;       // lambda_{n+1}: 27 planes of R, q = 0..26
  void *lam_out;            // lambda_n
  double *part;             // [gridDim.x] dJ/dsigmaT partials, accumulated
  double *dtw;              // [2][nx] dJ/dT_wall (bottom, top), accumulated
};

// ---- transpose of one site's collision -------------------------------------
// Inputs: the site's populations, its c (FP64) and stencil values, and lam
// (cotangents of the 27 post-collision values of the site).  Outputs: db, the
// cotangents of the 27 populations through this site's collision (including
// the paths through its own moments c, T, p, j); da, the cotangents of the
// seven stencil values (gcx, gcy, lapc, gTx, gTy, gpx, gpy), which stage B
// hands on to the neighbours' moments; and *dsT += dJ/dsigmaT.  The arithmetic
// differentiated is site_update's.
template <typename R, bool DEV>
__device__ __forceinline__ void site_adjoint(const StepArgs &a, const Consts<R> &k,
                                             const RowVals<R> &cur, double cd, R gcx, R gcy,
                                             R lapc, R gTx, R gTy, R gpx, R gpy, const R *lam,
                                             R *db, R *da, double *dsT) {
  const R third = R(1) / R(3);
  const R c = R(cd);
  // forward values
  R p = 0, jx = 0, jy = 0;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    p += cur.v[q];
    if (kEx[q] != 0) jx += R(kEx[q]) * cur.v[q];
    if (kEy[q] != 0) jy += R(kEy[q]) * cur.v[q];
  }
  double hs = 0.0;
#pragma unroll
  for (int q = 1; q < 9; ++q) hs += double(cur.v[18 + q]);
  const double Td = (cur.h0 + hs) / a.rcv;           // T, or Delta T
  const double Tfull_d = DEV ? Td + a.Ts : Td;
  const R Tv = R(Td), Tfull = R(Tfull_d);
  const R mu = R(a.beta2 * cd * (cd - 1.0) * (2.0 * cd - 1.0) - a.eps2 * double(lapc));
  const R Tm = R(Tfull_d - a.Tref);
  const R sigma = k.sigma0 - k.sigmaT * Tm;
  const R gsx = -k.sigmaT * gTx, gsy = -k.sigmaT * gTy;
  const R g2 = gcx * gcx + gcy * gcy;
  const R gds = gcx * gsx + gcy * gsy;
  const R ks = k.kcap * sigma * mu;
  const R ea = k.epsalpha;
  const R Fx = ks * gcx + ea * (g2 * gsx - gds * gcx) + k.bfx;
  const R Fy = ks * gcy + ea * (g2 * gsy - gds * gcy) + k.bfy;
  const R ux = R(3) * jx * k.inv_rho + R(0.5) * Fx * k.inv_rho;
  const R uy = R(3) * jy * k.inv_rho + R(0.5) * Fy * k.inv_rho;
  const bool inside = c > R(0) && c < R(1);
  const R ch = c < R(0) ? R(0) : (c > R(1) ? R(1) : c);
  const R wf = R(1) / (k.tauf0 + ch * k.dtauf);
  const R wT = R(1) / (k.tauT0 + ch * k.dtauT);
  const R wg = k.wg;
  const R Fbx = Fx - gpx, Fby = Fy - gpy;
  const R usq = ux * ux + uy * uy;
  const R rcvT = k.rcv * Tfull;
  const R cf = R(1) - R(0.5) * wf, cgf = R(1) - R(0.5) * wg, chf = R(1) - R(0.5) * wT;
  const R src_g = R(3) * c * k.inv_rho;
  const R src_h = R(3) * k.inv_rho;

  // reverse sweep over the nine directions (independent given the site
  // scalars, whose cotangents accumulate here)
  R b_wf = 0, b_wT = 0, b_p = 0, b_c = 0, b_gmu = 0, b_rcvT = 0, b_ux = 0, b_uy = 0;
  R b_Fx = 0, b_Fy = 0, b_Fbx = 0, b_Fby = 0, b_usq = 0, b_cf = 0, b_chf = 0, b_srcg = 0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const R w = wq<R>(i);
    const R e = R(kEx[i]) * ux + R(kEy[i]) * uy;
    const R G = w * (R(3) * e + R(4.5) * e * e - R(1.5) * usq);
    const R gam = w + G;
    const R cxu = R(kEx[i]) - ux, cyu = R(kEy[i]) - uy;
    const R fe = Fx * cxu + Fy * cyu;
    const R fbe = Fbx * cxu + Fby * cyu;
    const R Lf = lam[i], Lg = lam[9 + i], Lh = lam[18 + i];
    // f' = f - wf (f - feq) + cf fe gam,  feq = w p + rho/3 G
    const R feq = w * p + k.rho * third * G;
    db[i] = Lf * (R(1) - wf);
    b_wf -= Lf * (cur.v[i] - feq);
    const R b_feq = Lf * wf;
    b_cf += Lf * fe * gam;
    R b_fe = Lf * cf * gam;
    R b_gam = Lf * cf * fe;
    b_p += b_feq * w;
    R b_G = b_feq * k.rho * third;
    // g' = g - wg (g - geq) + cgf src_g fbe gam,
    // geq_0 = c - (1 - w0) gmu + c G_0, geq_i = w_i gmu + c G_i
    db[9 + i] = Lg * (R(1) - wg);
    const R b_geq = Lg * wg;
    b_srcg += Lg * cgf * fbe * gam;
    R b_fbe = Lg * cgf * src_g * gam;
    b_gam += Lg * cgf * src_g * fbe;
    b_c += b_geq * ((i == 0 ? R(1) : R(0)) + G);
    b_gmu += b_geq * (i == 0 ? -(R(1) - w) : w);
    b_G += b_geq * c;
    // h' = h - wT (h - heq) + chf src_h fbe heq,  heq = rho cv T gam
    R hd;   // h - heq
    if (i == 0) {
      hd = R(DEV ? cur.h0 - a.rcv * (Td * double(w) + Tfull_d * double(G))
                 : cur.h0 - a.rcv * Tfull_d * double(gam));
    } else {
      const R heq = DEV ? k.rcv * (Tv * w + Tfull * G) : rcvT * gam;
      hd = cur.v[18 + i] - heq;
    }
    const R heq_full = rcvT * gam;
    db[18 + i] = Lh * (R(1) - wT);
    b_wT -= Lh * hd;
    const R b_heq = Lh * (wT + chf * src_h * fbe);
    b_chf += Lh * src_h * fbe * heq_full;
    b_fbe += Lh * chf * src_h * heq_full;
    b_rcvT += b_heq * gam;
    b_gam += b_heq * rcvT;
    // gam = w + G,  G = w (3 e + 9/2 e^2 - 3/2 |u|^2)
    b_G += b_gam;
    const R b_e = b_G * w * (R(3) + R(9) * e);
    b_usq -= b_G * R(1.5) * w;
    b_ux += b_e * R(kEx[i]);
    b_uy += b_e * R(kEy[i]);
    b_Fx += b_fe * cxu;
    b_Fy += b_fe * cyu;
    b_Fbx += b_fbe * cxu;
    b_Fby += b_fbe * cyu;
    b_ux -= b_fe * Fx + b_fbe * Fbx;
    b_uy -= b_fe * Fy + b_fbe * Fby;
  }
  // site scalars
  b_wf -= R(0.5) * b_cf;
  b_wT -= R(0.5) * b_chf;
  b_c += b_srcg * R(3) * k.inv_rho;
  R b_mu = b_gmu * k.gam3;
  R b_T = b_rcvT * k.rcv;
  b_ux += R(2) * ux * b_usq;
  b_uy += R(2) * uy * b_usq;
  b_Fx += b_Fbx;
  b_Fy += b_Fby;
  const R b_gpx = -b_Fbx, b_gpy = -b_Fby;
  if (inside) b_c -= b_wf * wf * wf * k.dtauf + b_wT * wT * wT * k.dtauT;
  const R b_jx = b_ux * R(3) * k.inv_rho, b_jy = b_uy * R(3) * k.inv_rho;
  b_Fx += b_ux * R(0.5) * k.inv_rho;
  b_Fy += b_uy * R(0.5) * k.inv_rho;
  // F = ks grad c + ea (|grad c|^2 grad sigma - (grad c . grad sigma) grad c) + rho a
  const R b_ks = b_Fx * gcx + b_Fy * gcy;
  const R b_g2 = ea * (b_Fx * gsx + b_Fy * gsy);
  const R b_gds = -ea * (b_Fx * gcx + b_Fy * gcy);
  const R b_gcx = b_Fx * (ks - ea * gds) + b_gds * gsx + R(2) * gcx * b_g2;
  const R b_gcy = b_Fy * (ks - ea * gds) + b_gds * gsy + R(2) * gcy * b_g2;
  const R b_gsx = ea * g2 * b_Fx + b_gds * gcx;
  const R b_gsy = ea * g2 * b_Fy + b_gds * gcy;
  const R b_sigma = b_ks * k.kcap * mu;
  b_mu += b_ks * k.kcap * sigma;
  *dsT -= double(gTx) * double(b_gsx) + double(gTy) * double(b_gsy) + double(Tm) * double(b_sigma);
  b_T -= k.sigmaT * b_sigma;
  b_c += b_mu * R(a.beta2 * (6.0 * cd * cd - 6.0 * cd + 1.0));
  // own moments -> populations
  const R b_Tpop = b_T / k.rcv;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    db[q] += b_p + R(kEx[q]) * b_jx + R(kEy[q]) * b_jy;
    db[9 + q] += b_c;
    db[18 + q] += b_Tpop;
  }
  da[0] = b_gcx;
  da[1] = b_gcy;
  da[2] = -R(a.eps2) * b_mu;    // mu = mu0(c) - eps^2 lap c
  da[3] = -k.sigmaT * b_gsx;    // grad sigma = -sigmaT grad T
  da[4] = -k.sigmaT * b_gsy;
  da[5] = b_gpx;
  da[6] = b_gpy;
}

// ---- the adjoint step ---------------------------------------------------------
// Block: a strip of output columns [x0, x0 + nout); lane l runs stage A for
// column x0 - 1 + l (l <= nout + 1) and, for 1 <= l <= nout, stage B and the
// output of that column.  Moments span x0 - 2 .. x0 + nout + 1 (LDS position
// = column - x0 + 2).  Rows y0 - 1 .. y1 get stage A (the outer two only for
// their stencil cotangents), rows y0 .. y1 - 1 stage B.
template <typename R, bool DEV, int NW>
__global__ void __launch_bounds__(64 * NW)
adj_step_kernel(const AdjArgs aa) {
  constexpr int BX = 64 * NW;
  constexpr int WOUT = BX - 2;
  __shared__ double ringc[4][BX + 2];
  __shared__ R ringt[4][BX + 2];
  __shared__ R ringp[4][BX + 2];
  __shared__ R ringa[4][7][BX];
  __shared__ double red[NW];

  const StepArgs &a = aa.s;
  const int nx = a.nx, ny = a.ny;
  const bool walls = a.walls_y != 0;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int strip = tile % a.nstrips;
  const int chunk = tile / a.nstrips;
  const int x0 = strip * WOUT;
  const int nout = min(WOUT, nx - x0);
  const int lane = threadIdx.x;
  auto wrapx = [&](int v) {
    v %= nx;
    return v < 0 ? v + nx : v;
  };
  const int xa = wrapx(x0 - 1 + lane);
  const bool actA = lane <= nout + 1;
  const bool outl = lane >= 1 && lane <= nout;
  const int y0 = chunk * a.rows_per_chunk;
  const int y1 = min(y0 + a.rows_per_chunk, ny);
  const size_t n = (size_t)nx * (size_t)ny;
  const Consts<R> k(a);
  const double inv_rcv = 1.0 / a.rcv;
  using S = R;   // the state is stored in the arithmetic type

  const __amdgpu_buffer_rsrc_t rsrc = plane_rsrc(a.src, kNumS * n * sizeof(S) + 2 * n * 8);
  const uint32_t pbytes = (uint32_t)(n * sizeof(S));
  const uint32_t lbytes = (uint32_t)(n * sizeof(R));
  const __amdgpu_buffer_rsrc_t rin = plane_rsrc(aa.lam_in, 27 * n * sizeof(R));
  const __amdgpu_buffer_rsrc_t rout = plane_rsrc(aa.lam_out, 27 * n * sizeof(R));
  auto wrap_row = [&](int r) { return r < 0 ? r + ny : (r >= ny ? r - ny : r); };
  auto is_ghost = [&](int row) { return walls && (row < 0 || row >= ny); };
  auto load_vals = [&](int row, int col, RowVals<R> &r) {
    const uint32_t s = (uint32_t)(row * nx + col);
#pragma unroll
    for (int q = 0; q < 27; ++q)
      if (q != 9 && q != 18)
        r.v[q] = buf_load<S>(rsrc, s * (uint32_t)sizeof(S), (uint32_t)plane_of(q) * pbytes);
    r.g0 = buf_load<double>(rsrc, s * 8u, kNumS * pbytes);
    r.h0 = buf_load<double>(rsrc, s * 8u, kNumS * pbytes + (uint32_t)(n * 8));
  };
  auto lin = [&](int q, uint32_t s) {
    return buf_load<R>(rin, s * (uint32_t)sizeof(R), (uint32_t)q * lbytes);
  };

  // moments: lane l at LDS position l + 1; helpers (lanes 0, 1 of the last
  // wave) the columns x0 - 2 (position 0) and x0 + nout + 1 (position nout + 3)
  const int hl = lane - (BX - 64);
  const bool helper = hl == 0 || hl == 1;
  const int hcol = wrapx(hl == 0 ? x0 - 2 : x0 + nout + 1);
  const int hpos = hl == 0 ? 0 : nout + 3;
  auto put_one = [&](int slot, int rr, int col, int pos) {
    RowVals<R> r;
    load_vals(rr, col, r);
    double c, T;
    R p;
    site_moments(r, inv_rcv, &c, &T, &p);
    ringc[slot][pos] = c;
    ringt[slot][pos] = R(T);
    ringp[slot][pos] = p;
  };
  auto put_moments = [&](int row) {
    const int rr = wrap_row(row);
    if (actA) put_one(row & 3, rr, xa, lane + 1);
    if (helper) put_one(row & 3, rr, hcol, hpos);
  };
  // ghost row (halfway wall): c and p of the adjacent row, T = 2 T_wall - T
  auto put_ghost = [&](int row, int from) {
    const int s4 = row & 3, f4 = from & 3;
    const double *tw = row < 0 ? a.twb : a.twt;
    auto one = [&](int pos, int col) {
      ringc[s4][pos] = ringc[f4][pos];
      ringp[s4][pos] = ringp[f4][pos];
      const R twv = DEV ? R(tw[col] - a.Ts) : R(tw[col]);
      ringt[s4][pos] = R(2) * twv - ringt[f4][pos];
    };
    if (actA) one(lane + 1, xa);
    if (helper) one(hpos, hcol);
  };

  double dsT = 0.0;
  R dnew[27], dold[27];
#pragma unroll
  for (int q = 0; q < 27; ++q) dnew[q] = dold[q] = R(0);

  // stage A of row t
  auto stageA = [&](int t) {
    R *const aslot = &ringa[t & 3][0][lane];
    if (is_ghost(t) || !actA) {
#pragma unroll
      for (int m = 0; m < 7; ++m) aslot[m * BX] = R(0);
      return;
    }
    const bool own = outl && t >= y0 && t < y1;
    const int row = wrap_row(t);
    RowVals<R> cur;
    load_vals(row, xa, cur);
    // lambda* = Stream^T lambda_{n+1}
    R lam[27];
    const bool bot = walls && row == 0, top = walls && row == ny - 1;
    const uint32_t s_own = (uint32_t)(row * nx + xa);
    double tw_acc = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const bool out = (kEy[i] < 0 && bot) || (kEy[i] > 0 && top);
      if (out) {
        const int o = kOpp[i];
        lam[i] = lin(o, s_own);
        lam[9 + i] = lin(9 + o, s_own);
        const R lh = lin(18 + o, s_own);
        lam[18 + i] = -lh;
        tw_acc += 2.0 * double(wq<R>(i)) * a.rcv * double(lh);
      } else {
        const int xd = wrapx(xa + kEx[i]);
        const int yd = wrap_row(row + kEy[i]);
        const uint32_t s = (uint32_t)(yd * nx + xd);
        lam[i] = lin(i, s);
        lam[9 + i] = lin(9 + i, s);
        lam[18 + i] = lin(18 + i, s);
      }
    }
    if (own && (bot || top)) aa.dtw[(bot ? 0 : nx) + xa] += tw_acc;
    // stencils at (xa, t), as in the forward step
    const int l = lane;
    const double *cS = &ringc[(t - 1) & 3][l], *cC = &ringc[t & 3][l];
    const double *cN = &ringc[(t + 1) & 3][l];
    const R *tS = &ringt[(t - 1) & 3][l], *tC = &ringt[t & 3][l], *tN = &ringt[(t + 1) & 3][l];
    const R *pS = &ringp[(t - 1) & 3][l], *pC = &ringp[t & 3][l], *pN = &ringp[(t + 1) & 3][l];
    const double cd = cC[1];
    double gcx_d, gcy_d, lap_d;
    {
      const double e = cC[2], w = cC[0], nn = cN[1], s = cS[1];
      const double ne = cN[2], nw = cN[0], sw = cS[0], se = cS[2];
      gcx_d = (e - w) * (1.0 / 3.0) + (ne + se - nw - sw) * (1.0 / 12.0);
      gcy_d = (nn - s) * (1.0 / 3.0) + (ne + nw - se - sw) * (1.0 / 12.0);
      lap_d = (2.0 / 3.0) * ((e - cd) + (w - cd) + (nn - cd) + (s - cd)) +
              (1.0 / 6.0) * ((ne - cd) + (nw - cd) + (se - cd) + (sw - cd));
    }
    const R third = R(1) / R(3);
    auto grad = [&](const R *Sr, const R *Cr, const R *Nr, R *gx, R *gy) {
      *gx = (Cr[2] - Cr[0]) * third + (Nr[2] + Sr[2] - Nr[0] - Sr[0]) * R(1.0 / 12.0);
      *gy = (Nr[1] - Sr[1]) * third + (Nr[2] + Nr[0] - Sr[2] - Sr[0]) * R(1.0 / 12.0);
    };
    R gTx, gTy, gpx, gpy;
    grad(tS, tC, tN, &gTx, &gTy);
    grad(pS, pC, pN, &gpx, &gpy);
    R da[7];
    double ds = 0.0;
    site_adjoint<R, DEV>(a, k, cur, cd, R(gcx_d), R(gcy_d), R(lap_d), gTx, gTy, gpx, gpy, lam,
                         dnew, da, &ds);
#pragma unroll
    for (int m = 0; m < 7; ++m) aslot[m * BX] = da[m];
    if (own) dsT += ds;
  };

  // stage B of row t (a real row of the chunk); dold holds its direct part
  auto stageB = [&](int t) {
    if (!outl) return;
    const int l = lane;
    R cb = 0, Tb = 0, pb = 0;
    // x = y - xi_k reads y through direction k of its stencil
#pragma unroll
    for (int kk = 1; kk < 9; ++kk) {
      const int xr = t - kEy[kk];
      if (is_ghost(xr)) continue;
      const R *ar = &ringa[xr & 3][0][l - kEx[kk]];
      const R wk = wq<R>(kk);
      const R gx = R(3) * wk * R(kEx[kk]), gy = R(3) * wk * R(kEy[kk]);
      cb += gx * ar[0] + gy * ar[BX] + R(6) * wk * ar[2 * BX];
      Tb += gx * ar[3 * BX] + gy * ar[4 * BX];
      pb += gx * ar[5 * BX] + gy * ar[6 * BX];
    }
    cb -= R(10.0 / 3.0) * ringa[t & 3][2][l];   // centre weight of the Laplacian
    // wall rows: x in the same row whose stencil direction k points into the
    // ghost row reads the mirror image of x + xi_k, which is y
    if (walls && (t == 0 || t == ny - 1)) {
      const int dir = t == 0 ? -1 : 1;
      double twb = 0.0;
#pragma unroll
      for (int kk = 1; kk < 9; ++kk) {
        if (kEy[kk] != dir) continue;
        const R *ar = &ringa[t & 3][0][l - kEx[kk]];
        const R wk = wq<R>(kk);
        const R gx = R(3) * wk * R(kEx[kk]), gy = R(3) * wk * R(kEy[kk]);
        cb += gx * ar[0] + gy * ar[BX] + R(6) * wk * ar[2 * BX];
        pb += gx * ar[5 * BX] + gy * ar[6 * BX];
        const R tg = gx * ar[3 * BX] + gy * ar[4 * BX];
        Tb -= tg;
        twb += 2.0 * double(tg);
      }
      aa.dtw[(t == 0 ? 0 : nx) + xa] += twb;
    }
    const uint32_t s = (uint32_t)(t * nx + xa);
    const R Tpop = Tb * R(inv_rcv);
#pragma unroll
    for (int q = 0; q < 27; ++q) {
      const R add = q < 9 ? pb : (q < 18 ? cb : Tpop);
      buf_store_nt<R>(dold[q] + add, rout, s * (uint32_t)sizeof(R), (uint32_t)q * lbytes);
    }
  };

  // prologue: rows y0 - 2 and y0 - 1 (a ghost row after its real neighbour)
  {
    const int r2 = y0 - 2, r1 = y0 - 1;
    if (!is_ghost(r1)) put_moments(r1);
    if (!is_ghost(r2)) put_moments(r2);
    else if (!is_ghost(r1)) put_ghost(r2, r1);
  }
  for (int t = y0 - 1; t <= y1; ++t) {
    const int tn = t + 1;
    if (!is_ghost(tn)) put_moments(tn);
    else if (!is_ghost(t)) put_ghost(tn, t);
    if (t == y0 - 1 && is_ghost(t) && !is_ghost(tn)) put_ghost(t, tn);
    __syncthreads();
    stageA(t);
    __syncthreads();
    if (t - 1 >= y0) stageB(t - 1);
#pragma unroll
    for (int q = 0; q < 27; ++q) dold[q] = dnew[q];
  }
  // dJ/dsigmaT: deterministic block sum, accumulated over the steps
  {
    const int wave = lane >> 6, wl = lane & 63;
    double v = dsT;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (wl == 0) red[wave] = v;
    __syncthreads();
    if (lane == 0) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) sum += red[w];
      aa.part[blockIdx.x] += sum;
    }
  }
}

// lambda_N from the seed on c = sum_q g_q: the seed on each g_q.
template <typename R>
__global__ void __launch_bounds__(256)
adj_seed_kernel(R *__restrict__ lam, const double *__restrict__ dJdc, size_t n) {
  const size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (s >= n) return;
  lam[q * n + s] = (q >= 9 && q < 18) ? R(dJdc[s]) : R(0);
}

// lambda_0 -> FP64 outputs: dJ/dF_0 (optional) and dJ/dT_0 through the initial
// equilibrium hbar_i = w_i rho cv T_0 (optional).
template <typename R>
__global__ void __launch_bounds__(256)
adj_finish_kernel(const R *__restrict__ lam, double *__restrict__ dF0, double *__restrict__ dT0,
                  size_t n, double rcv) {
  const size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    const double v = double(lam[q * n + s]);
    if (dF0) dF0[q * n + s] = v;
    if (q >= 18) t += wq<double>(q - 18) * rcv * v;
  }
  if (dT0) dT0[s] = t;
}

// fixed-order sum of the per-block partials
__global__ void __launch_bounds__(256)
adj_sum_kernel(const double *__restrict__ part, int nb, double *__restrict__ out) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) acc += part[b];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

__global__ void __launch_bounds__(256)
adj_zero_kernel(double *__restrict__ p, size_t count) {
  const size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < count) p[s] = 0.0;
}

}  // namespace lbe
