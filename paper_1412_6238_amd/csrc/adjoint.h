// adjoint.h -- reverse-mode differentiation of the fused step: checkpoint
// layout, the adjoint step kernels and their helpers.
//
// One step is F_{n+1} = Stream(Collide(F_n)).  Collide at site x depends on
// F_n(x) and, through the nine-point stencils, on the moments (c, T, p) of the
// eight neighbours.  For a cotangent lambda_{n+1} of F_{n+1} the adjoint step
// returns lambda_n = (dF_{n+1}/dF_n)^T lambda_{n+1}.  The cotangent is kept
// in two parts, lambda_q = D_q + M_{group(q)}: D holds 27 planes and M three
// (the shares of p = sum f, c = sum g and rho cv T = sum hbar, which reach
// every population of a group alike).  One adjoint step is two kernels, one
// thread per site, no recomputation:
//   adj_collide_kernel  lambda* = Stream^T lambda_{n+1}, a pull from x + xi_i
//       (at a wall the reflected population of the same site, with the sign
//       flip of the anti-bounce-back for hbar, whose wall term 2 w rho cv
//       T_wall gives dJ/dT_wall); then the transpose of the site's collision
//       (site_adjoint): D_n(x), the stencil cotangents A_n(x) (grad c, lap c,
//       grad T, grad p) and the site's share of dJ/dsigmaT;
//   adj_stencil_kernel  the stencil transposes: the moments of site y collect
//       A_n(x) from every x whose stencil reads y (in the wall rows the ghost
//       row mirrors c and p and holds 2 T_wall - T, so T collects with a minus
//       sign and T_wall twice) into M_n(y).
// The linearisation point (c, T, p, j of F_n) comes from a moment tape that
// the replay writes; the populations themselves are read only when the
// relaxation times vary with c.
//
// The plane sets D (27 planes), M (3) and A (7, or 10 with the curvature
// form) are row-interleaved like the state: plane p of site (x, y) in a set
// of P planes sits at element (y P + p) nx + x (adj_index), so that a row of
// tiles reads and writes one stretch of memory per row.
//
// The run is differentiated by sqrt(N) checkpointing: the forward run saves
// every K-th state (K = ceil(sqrt N)); the backward pass replays each segment
// from its checkpoint, writing the moment tape (and, with c-dependent
// relaxation times, keeping the states), and sweeps it in reverse.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "step_kernel.h"

namespace lbe {

inline int adj_save_checkpoint(char *adj_base, const AdjLayout &A, int64_t k,
                               const void *state, size_t bytes, hipStream_t st) {
  if (k < 0 || k >= A.nchk) return 1;
  char *dst = adj_base + A.off_chk + (size_t)k * A.state_bytes;
  return hipMemcpyAsync(dst, state, bytes, hipMemcpyDeviceToDevice, st) == hipSuccess ? 0 : 1;
}

// element of plane p at (x, y) in a row-interleaved set of P planes
__host__ __device__ __forceinline__ size_t adj_index(int P, int p, size_t nx, size_t y,
                                                     size_t x) {
  return (y * (size_t)P + (size_t)p) * nx + x;
}

struct AdjArgs {
  StepArgs s;          // constants; s.tape = moments of F_n, s.src = F_n (VARTAU)
  const void *d_in;    // D_{n+1}: 27 planes of R
  const void *m_in;    // M_{n+1}: 3 planes of R (f, g, hbar groups)
  void *d_out;         // D_n
  void *a;             // A_n: kAdjA planes of R (collide writes, stencil reads)
  void *m_out;         // M_n
  double *part;        // [tiles] dJ/dsigmaT partials, accumulated over steps
  double *dtw;         // [2][nx] dJ/dT_wall (bottom, top), accumulated
  int ntx;             // tiles along x
};

// ---- transpose of one site's collision -------------------------------------
// Inputs: the site's moments (p, j, T or their deviations; c in FP64), its
// stencil values, lam (cotangents of the 27 post-collision values of the site)
// and, when the relaxation times vary with c (VARTAU), its populations.
// Outputs: db, the cotangents of the 27 populations through this site's
// collision (including the paths through its own moments c, T, p, j); da, the
// cotangents of the stencil values (gcx, gcy, lapc, gTx, gTy, gpx, gpy, and
// with CURV the Hessian hxx, hxy, hyy of the curvature form), which the
// stencil transpose hands on to the neighbours' moments; and
// *dsT += dJ/dsigmaT.  The arithmetic differentiated is site_update's.  With
// constant relaxation times the populations enter the collision only through
// the moments, so the moments suffice.
template <typename R, bool DEV, bool VARTAU, bool CURV>
__device__ __forceinline__ void site_adjoint(const StepArgs &a, const Consts<R> &k,
                                             const RowVals<R> &cur, R p, R jx, R jy, double Td,
                                             double Trow, double cd, R gcx, R gcy, R lapc,
                                             R gTx, R gTy, R gpx, R gpy, R hxx, R hxy, R hyy,
                                             const R *lam, R *db, R *da, double *dsT) {
  const R third = R(1) / R(3);
  const R c = R(cd);
  const double Tfull_d = DEV ? Td + Trow : Td;
  const R Tv = R(Td), Tfull = R(Tfull_d);
  const R mu = R(a.beta2 * cd * (cd - 1.0) * (2.0 * cd - 1.0) - a.eps2 * double(lapc));
  const R Tm = R(Tfull_d - a.Tref);
  const R sigma = k.sigma0 - k.sigmaT * Tm;
  const R gsx = -k.sigmaT * gTx, gsy = -k.sigmaT * gTy;
  const R g2 = gcx * gcx + gcy * gcy;
  const R gds = gcx * gsx + gcy * gsy;
  const R ea = k.epsalpha;
  // capillary coefficient along grad c: kcap sigma mu (potential form) or
  // -sigma eps alpha t.H.t (curvature form, t.H.t = N / |grad c|^2)
  const R Nh = gcy * gcy * hxx - R(2) * gcx * gcy * hxy + gcx * gcx * hyy;
  const R tHt = (CURV && g2 > R(0)) ? Nh / g2 : R(0);
  const R ks = CURV ? -sigma * ea * tHt : k.kcap * sigma * mu;
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
    if (VARTAU) b_wf -= Lf * (cur.v[i] - feq);
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
    if (VARTAU) {
      R hd;   // h - heq
      if (i == 0) {
        hd = R(DEV ? cur.h0() - a.rcv * (Td * double(w) + Tfull_d * double(G))
                   : cur.h0() - a.rcv * Tfull_d * double(gam));
      } else {
        const R heq = DEV ? k.rcv * (Tv * w + Tfull * G) : rcvT * gam;
        hd = cur.v[18 + i] - heq;
      }
      b_wT -= Lh * hd;
    }
    const R heq_full = rcvT * gam;
    db[18 + i] = Lh * (R(1) - wT);
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
  if (VARTAU && inside) b_c -= b_wf * wf * wf * k.dtauf + b_wT * wT * wT * k.dtauT;
  const R b_jx = b_ux * R(3) * k.inv_rho, b_jy = b_uy * R(3) * k.inv_rho;
  b_Fx += b_ux * R(0.5) * k.inv_rho;
  b_Fy += b_uy * R(0.5) * k.inv_rho;
  // F = ks grad c + ea (|grad c|^2 grad sigma - (grad c . grad sigma) grad c) + rho a
  const R b_ks = b_Fx * gcx + b_Fy * gcy;
  const R b_g2 = ea * (b_Fx * gsx + b_Fy * gsy);
  const R b_gds = -ea * (b_Fx * gcx + b_Fy * gcy);
  R b_gcx = b_Fx * (ks - ea * gds) + b_gds * gsx + R(2) * gcx * b_g2;
  R b_gcy = b_Fy * (ks - ea * gds) + b_gds * gsy + R(2) * gcy * b_g2;
  const R b_gsx = ea * g2 * b_Fx + b_gds * gcx;
  const R b_gsy = ea * g2 * b_Fy + b_gds * gcy;
  R b_sigma, b_hxx = 0, b_hxy = 0, b_hyy = 0;
  if (CURV) {
    // ks = -sigma ea tHt, tHt = N / g2 with N = gy^2 hxx - 2 gx gy hxy + gx^2 hyy
    b_sigma = -b_ks * ea * tHt;
    if (g2 > R(0)) {
      const R b_t = -b_ks * sigma * ea;
      const R ig2 = R(1) / g2;
      b_hxx = b_t * gcy * gcy * ig2;
      b_hyy = b_t * gcx * gcx * ig2;
      b_hxy = -b_t * R(2) * gcx * gcy * ig2;
      b_gcx += b_t * ((R(2) * gcx * hyy - R(2) * gcy * hxy) - R(2) * gcx * tHt) * ig2;
      b_gcy += b_t * ((R(2) * gcy * hxx - R(2) * gcx * hxy) - R(2) * gcy * tHt) * ig2;
    }
  } else {
    b_sigma = b_ks * k.kcap * mu;
    b_mu += b_ks * k.kcap * sigma;
  }
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
  if (CURV) {
    da[7] = b_hxx;
    da[8] = b_hxy;
    da[9] = b_hyy;
  }
}


// ---- adjoint step, part 1: pull and collision transpose ----------------------
template <typename R, bool DEV, bool VARTAU, bool CURV>
__global__ void __launch_bounds__(kAdjTX * kAdjTY)
adj_collide_kernel(const AdjArgs aa) {
  constexpr int TW = kAdjTX + 2, TH = kAdjTY + 2;
  __shared__ double lc[TH][TW];
  __shared__ R lt[TH][TW];
  __shared__ R lp[TH][TW];
  __shared__ double red[kAdjTX * kAdjTY / 64];

  const StepArgs &a = aa.s;
  const int nx = a.nx, ny = a.ny;
  const bool walls = a.walls_y != 0;
  const size_t n = (size_t)nx * (size_t)ny;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % aa.ntx) * kAdjTX, y0 = (tile / aa.ntx) * kAdjTY;
  const int tid = threadIdx.x;
  const double *tape_c = static_cast<const double *>(a.tape);
  const R *tape_r = reinterpret_cast<const R *>(tape_c + n);
  auto wrapx = [&](int v) {
    v %= nx;
    return v < 0 ? v + nx : v;
  };
  auto wrapy = [&](int v) {
    v %= ny;
    return v < 0 ? v + ny : v;
  };

  // moments of the tile and its one-site halo; ghost rows beyond a wall
  // mirror c and p and hold T_ghost = 2 T_wall - T (deviations: 2 (T_wall -
  // Ts) - Delta T)
  for (int e = tid; e < TH * TW; e += kAdjTX * kAdjTY) {
    const int r = e / TW, q = e - r * TW;
    const int row = y0 - 1 + r, col = wrapx(x0 - 1 + q);
    if (walls && (row < 0 || row >= ny)) {
      const size_t s = (size_t)(row < 0 ? 0 : ny - 1) * nx + col;
      const double *tw = row < 0 ? a.twb : a.twt;
      const double twref = DEV ? a.Ts + (row < 0 ? 0.0 : a.Tg * double(ny)) : 0.0;
      const R twv = DEV ? R(tw[col] - twref) : R(tw[col]);
      lc[r][q] = tape_c[s];
      lp[r][q] = tape_r[n + s];
      lt[r][q] = R(2) * twv - tape_r[s];
    } else {
      const size_t s = (size_t)wrapy(row) * nx + col;
      lc[r][q] = tape_c[s];
      lt[r][q] = tape_r[s];
      lp[r][q] = tape_r[n + s];
    }
  }
  __syncthreads();

  const int lx = tid & (kAdjTX - 1), ly = tid / kAdjTX;
  const int x = x0 + lx, y = y0 + ly;
  double ds = 0.0;
  if (x < nx && y < ny) {
    const Consts<R> k(a);
    const uint32_t s = (uint32_t)(y * nx + x);
    constexpr uint32_t E = sizeof(R);
    const uint32_t seg = (uint32_t)nx * E;   // one plane's segment of a row
    const __amdgpu_buffer_rsrc_t rd = plane_rsrc(aa.d_in, 27 * n * sizeof(R));
    const __amdgpu_buffer_rsrc_t rm = plane_rsrc(aa.m_in, 3 * n * sizeof(R));
    auto ldD = [&](int q, int yy, int xx) {
      return buf_load<R>(rd, (uint32_t)yy * 27u * seg + (uint32_t)xx * E, (uint32_t)q * seg);
    };
    auto ldM = [&](int g, int yy, int xx) {
      return buf_load<R>(rm, (uint32_t)yy * 3u * seg + (uint32_t)xx * E, (uint32_t)g * seg);
    };
    // lambda* = Stream^T lambda_{n+1}
    R lam[27];
    const bool bot = walls && y == 0, top = walls && y == ny - 1;
    double tw_acc = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const bool out = (kEy[i] < 0 && bot) || (kEy[i] > 0 && top);
      int sy = y, sx = x;
      int dq = i;
      if (out) {
        dq = kOpp[i];
      } else if (i != 0) {
        sy = wrapy(y + kEy[i]);
        sx = wrapx(x + kEx[i]);
      }
      lam[i] = ldD(dq, sy, sx) + ldM(0, sy, sx);
      lam[9 + i] = ldD(9 + dq, sy, sx) + ldM(1, sy, sx);
      const R lh = ldD(18 + dq, sy, sx) + ldM(2, sy, sx);
      if (out) {
        lam[18 + i] = -lh;
        tw_acc += 2.0 * double(wq<R>(i)) * a.rcv * double(lh);
      } else {
        lam[18 + i] = lh;
      }
    }
    if (bot || top) aa.dtw[(bot ? 0 : nx) + x] += tw_acc;
    // linearisation point and stencils, as in the forward step
    const int cx = lx + 1, cy = ly + 1;
    const double cd = lc[cy][cx];
    double gcx_d, gcy_d, lap_d, hxx_d = 0.0, hxy_d = 0.0, hyy_d = 0.0;
    {
      const double e = lc[cy][cx + 1], w = lc[cy][cx - 1], nn = lc[cy + 1][cx],
                   so = lc[cy - 1][cx];
      const double ne = lc[cy + 1][cx + 1], nw = lc[cy + 1][cx - 1], sw = lc[cy - 1][cx - 1],
                   se = lc[cy - 1][cx + 1];
      gcx_d = (e - w) * (1.0 / 3.0) + (ne + se - nw - sw) * (1.0 / 12.0);
      gcy_d = (nn - so) * (1.0 / 3.0) + (ne + nw - se - sw) * (1.0 / 12.0);
      const double dx2 = (e - cd) + (w - cd), dy2 = (nn - cd) + (so - cd);
      const double dd = (ne - cd) + (nw - cd) + (se - cd) + (sw - cd);
      lap_d = (2.0 / 3.0) * (dx2 + dy2) + (1.0 / 6.0) * dd;
      if (CURV) {
        hxx_d = (2.0 / 3.0) * dx2 - (1.0 / 3.0) * dy2 + (1.0 / 6.0) * dd;
        hyy_d = (2.0 / 3.0) * dy2 - (1.0 / 3.0) * dx2 + (1.0 / 6.0) * dd;
        hxy_d = 0.25 * ((ne - nw) - (se - sw));
      }
    }
    const R third = R(1) / R(3);
    auto grad = [&](R (*f)[TW], R *gx, R *gy) {
      *gx = (f[cy][cx + 1] - f[cy][cx - 1]) * third +
            (f[cy + 1][cx + 1] + f[cy - 1][cx + 1] - f[cy + 1][cx - 1] - f[cy - 1][cx - 1]) *
                R(1.0 / 12.0);
      *gy = (f[cy + 1][cx] - f[cy - 1][cx]) * third +
            (f[cy + 1][cx + 1] + f[cy + 1][cx - 1] - f[cy - 1][cx + 1] - f[cy - 1][cx - 1]) *
                R(1.0 / 12.0);
    };
    R gTx, gTy, gpx, gpy;
    grad(lt, &gTx, &gTy);
    grad(lp, &gpx, &gpy);
    if (DEV) gTy += R(a.Tg);   // linear temperature reference of the FP32 form
    const double Trow = DEV ? a.Ts + a.Tg * (double(y) + 0.5) : 0.0;
    RowVals<R> cur;
    if (VARTAU) {
      const __amdgpu_buffer_rsrc_t rs =
          plane_rsrc(a.src, state_bytes_for<R>(n));
      const uint32_t ro = (uint32_t)y * (uint32_t)row_bytes<R>(nx);
      const uint32_t segb = (uint32_t)(nx * sizeof(R));   // a plane's segment of a row
#pragma unroll
      for (int q = 0; q < 27; ++q)
        if (q != 9 && q != 18)
          cur.v[q] = buf_load<R>(rs, ro + (uint32_t)x * (uint32_t)sizeof(R),
                                 (uint32_t)plane_of(q) * segb);
      cur.g0r = rest_load_raw<R, 0>(rs, ro, x, (uint32_t)rest_base<R>(0, nx));
      cur.h0r = rest_load_raw<R, 1>(rs, ro, x, (uint32_t)rest_base<R>(1, nx));
    }
    constexpr int NA = CURV ? kAdjA : 7;
    R db[27], da[kAdjA];
    site_adjoint<R, DEV, VARTAU, CURV>(a, k, cur, lp[cy][cx], tape_r[2 * n + s],
                                       tape_r[3 * n + s], double(lt[cy][cx]), Trow, cd,
                                       R(gcx_d), R(gcy_d), R(lap_d), gTx, gTy, gpx, gpy,
                                       R(hxx_d), R(hxy_d), R(hyy_d), lam, db, da, &ds);
    const __amdgpu_buffer_rsrc_t wd = plane_rsrc(aa.d_out, 27 * n * sizeof(R));
    const __amdgpu_buffer_rsrc_t wa = plane_rsrc(aa.a, kAdjA * n * sizeof(R));
#pragma unroll
    for (int q = 0; q < 27; ++q)
      buf_store<R>(db[q], wd, (uint32_t)y * 27u * seg + (uint32_t)x * E, (uint32_t)q * seg);
#pragma unroll
    for (int m = 0; m < NA; ++m)
      buf_store<R>(da[m], wa, (uint32_t)y * (uint32_t)NA * seg + (uint32_t)x * E,
                   (uint32_t)m * seg);
  }
  // dJ/dsigmaT: deterministic block sum, accumulated over the steps
  {
    const int wave = tid >> 6;
    double v = ds;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((tid & 63) == 0) red[wave] = v;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < kAdjTX * kAdjTY / 64; ++w) sum += red[w];
      aa.part[blockIdx.x] += sum;
    }
  }
}

// ---- adjoint step, part 2: stencil transposes --------------------------------
// weight of neighbour direction k in the Hessian stencil of c, applied to the
// cotangents (a_xx, a_xy, a_yy) of the site reading it: w_k (9 xi_x^2 - 3),
// 9 w_k xi_x xi_y and w_k (9 xi_y^2 - 3)
template <typename R>
__device__ __forceinline__ R hess_w(int kk, R axx, R axy, R ayy) {
  const R wk = wq<R>(kk);
  const R ex = R(kEx[kk]), ey = R(kEy[kk]);
  return wk * ((R(9) * ex * ex - R(3)) * axx + R(9) * ex * ey * axy + (R(9) * ey * ey - R(3)) * ayy);
}


template <typename R, bool CURV>
__global__ void __launch_bounds__(kAdjTX * kAdjTY)
adj_stencil_kernel(const AdjArgs aa) {
  constexpr int TW = kAdjTX + 2, TH = kAdjTY + 2;
  constexpr int NA = CURV ? kAdjA : 7;
  __shared__ R la[NA][TH][TW];

  const StepArgs &a = aa.s;
  const int nx = a.nx, ny = a.ny;
  const bool walls = a.walls_y != 0;
  const size_t n = (size_t)nx * (size_t)ny;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % aa.ntx) * kAdjTX, y0 = (tile / aa.ntx) * kAdjTY;
  const int tid = threadIdx.x;
  constexpr uint32_t E = sizeof(R);
  const uint32_t seg = (uint32_t)nx * E;   // one plane's segment of a row
  const __amdgpu_buffer_rsrc_t ra = plane_rsrc(aa.a, kAdjA * n * sizeof(R));
  auto wrapx = [&](int v) {
    v %= nx;
    return v < 0 ? v + nx : v;
  };
  auto wrapy = [&](int v) {
    v %= ny;
    return v < 0 ? v + ny : v;
  };
  auto ghost = [&](int row) { return walls && (row < 0 || row >= ny); };
  for (int e = tid; e < TH * TW; e += kAdjTX * kAdjTY) {
    const int r = e / TW, q = e - r * TW;
    const int row = y0 - 1 + r;
    if (ghost(row)) {
#pragma unroll
      for (int m = 0; m < NA; ++m) la[m][r][q] = R(0);   // no stencil at a ghost site
    } else {
      const uint32_t off = (uint32_t)wrapy(row) * (uint32_t)NA * seg + (uint32_t)wrapx(x0 - 1 + q) * E;
#pragma unroll
      for (int m = 0; m < NA; ++m) la[m][r][q] = buf_load<R>(ra, off, (uint32_t)m * seg);
    }
  }
  __syncthreads();
  const int lx = tid & (kAdjTX - 1), ly = tid / kAdjTX;
  const int x = x0 + lx, y = y0 + ly;
  if (x >= nx || y >= ny) return;
  const int cx = lx + 1, cy = ly + 1;
  R cb = 0, Tb = 0, pbv = 0;
  // site x = y - xi_k reads y through direction k of its stencil
#pragma unroll
  for (int kk = 1; kk < 9; ++kk) {
    const int r = cy - kEy[kk], q = cx - kEx[kk];
    const R wk = wq<R>(kk);
    const R gx = R(3) * wk * R(kEx[kk]), gy = R(3) * wk * R(kEy[kk]);
    cb += gx * la[0][r][q] + gy * la[1][r][q] + R(6) * wk * la[2][r][q];
    Tb += gx * la[3][r][q] + gy * la[4][r][q];
    pbv += gx * la[5][r][q] + gy * la[6][r][q];
    if constexpr (CURV) cb += hess_w(kk, la[7][r][q], la[8][r][q], la[9][r][q]);
  }
  cb -= R(10.0 / 3.0) * la[2][cy][cx];   // centre weight of the Laplacian
  if constexpr (CURV) cb -= R(4.0 / 3.0) * (la[7][cy][cx] + la[9][cy][cx]);   // of hxx, hyy
  // wall rows: a site x of the same row whose stencil direction k points into
  // the ghost row reads the mirror image of x + xi_k, which is y
  if (walls && (y == 0 || y == ny - 1)) {
    const int dir = y == 0 ? -1 : 1;
    double twb = 0.0;
#pragma unroll
    for (int kk = 1; kk < 9; ++kk) {
      if (kEy[kk] != dir) continue;
      const int q = cx - kEx[kk];
      const R wk = wq<R>(kk);
      const R gx = R(3) * wk * R(kEx[kk]), gy = R(3) * wk * R(kEy[kk]);
      cb += gx * la[0][cy][q] + gy * la[1][cy][q] + R(6) * wk * la[2][cy][q];
      if constexpr (CURV) cb += hess_w(kk, la[7][cy][q], la[8][cy][q], la[9][cy][q]);
      pbv += gx * la[5][cy][q] + gy * la[6][cy][q];
      const R tg = gx * la[3][cy][q] + gy * la[4][cy][q];
      Tb -= tg;
      twb += 2.0 * double(tg);
    }
    aa.dtw[(y == 0 ? 0 : nx) + x] += twb;
  }
  const uint32_t off = (uint32_t)y * 3u * seg + (uint32_t)x * E;
  const __amdgpu_buffer_rsrc_t wm = plane_rsrc(aa.m_out, 3 * n * sizeof(R));
  buf_store<R>(pbv, wm, off, 0u);
  buf_store<R>(cb, wm, off, seg);
  buf_store<R>(Tb * R(1.0 / a.rcv), wm, off, 2 * seg);
}

// lambda_N from the seed on c = sum_q g_q: D = the seed on each g_q, M = 0.
template <typename R>
__global__ void __launch_bounds__(256)
adj_seed_kernel(R *__restrict__ d, R *__restrict__ m, const double *__restrict__ dJdc,
                size_t n, size_t nx) {
  const size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (s >= n) return;
  const size_t y = s / nx, x = s - y * nx;
  d[adj_index(27, q, nx, y, x)] = (q >= 9 && q < 18) ? R(dJdc[s]) : R(0);
  if (q < 3) m[adj_index(3, q, nx, y, x)] = R(0);
}

// lambda_0 = D_0 + M_0 -> FP64 outputs: dJ/dF_0 (optional) and dJ/dT_0 through
// the initial equilibrium hbar_i = w_i rho cv T_0 (optional).
template <typename R>
__global__ void __launch_bounds__(256)
adj_finish_kernel(const R *__restrict__ d, const R *__restrict__ m, double *__restrict__ dF0,
                  double *__restrict__ dT0, size_t n, size_t nx, double rcv) {
  const size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const size_t y = s / nx, x = s - y * nx;
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    const double v = double(d[adj_index(27, q, nx, y, x)]) + double(m[adj_index(3, q / 9, nx, y, x)]);
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
