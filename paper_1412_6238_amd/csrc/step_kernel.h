// step_kernel.h -- the fused CSF lattice Boltzmann step on gfx950.
//
// One launch performs, for every site, the whole step of arXiv:1412.6238:
//   moments      c = sum g (Eq. 15), rho cv T = sum hbar (Eq. 26),
//                p = sum f, j = sum xi f                  (Eq. 9)
//   stencils     grad c, lap c, grad T, grad p (isotropic nine-point; wall
//                ghosts: c and p mirrored, T_ghost = 2 T_wall - T)
//   closures     mu = mu0(c) - eps^2 lap c (Eq. 16), sigma(T) (Eq. 5),
//                CSF force F (Eqs. 3-4, capillary part in the potential form,
//                or with kCurv in the curvature form), u (Eq. 9 with the
//                half force (1/2) cs^2 F), relaxation rates, Fbar = F - grad p
//   collisions   f (Eqs. 6-8), g (Eqs. 12-14), hbar (Eqs. 22, 25)
//   streaming    push to x + xi (x periodic); halfway bounce-back for f, g
//                and anti-bounce-back with the wall temperature for hbar
//
// State layout (row-interleaved, x fastest; host_layout.h): each row holds
// the row's segment of each of 25 planes of the storage type S -- f_0..8,
// g_1..8, hbar_1..8 -- then those of the rest populations g_0 and hbar_0.
// The rest populations carry the two transported scalars (c = g_0 +
// small terms, rho cv T = hbar_0 + eight smaller terms).  g_0 stays FP64 in
// both forms, which keeps c accurate to far below FP32 rounding (c enters
// the force through eps^2 lap c); the FP32 form holds hbar_0 as an FP32
// deviation.  The FP32 form therefore moves 2 x (26 x 4 + 8) = 224 bytes per
// site update, against the 216 of 27 FP32 values.
//
// The state held is F_n (pre-collision).  A lane reads the 27 values of its
// own site (coalesced, aligned) and pushes post-collision values to the
// neighbours' slots in the other buffer (shifted by at most one element).
//
// Work decomposition: a block owns a strip of 64*NW columns and marches up a
// chunk of rows, one column per lane.  The moments a row's stencils need
// (c, T, p) sit in an LDS ring of four rows, filled one row ahead of the row
// being collided; helper lanes add the halo column on each side.  PIPE 2
// issues the loads of a row two rows ahead of its collision and keeps two
// rows in registers; PIPE 1 keeps the next row's values in registers,
// loaded one row ahead of the collision; PIPE 0 loads a row twice (for the
// moments and again, from cache, for the collision).
// Every distribution is read from HBM once per step (halo columns and the
// two boundary rows of a chunk are read again by the neighbouring block).
//
// Mode bits (template MODE): kStore (collide and stream), kDiag (FP64
// diagnostic partials), kFields (macroscopic output), kTape (moments for the
// adjoint), kCurv (capillary force in the curvature form of Eq. 4), kVarRho
// (two densities; the ring then holds the pressure of Eq. 9, which a
// kVarRho | kPress launch of the same kernel writes first), kStream (whole-line
// stores bypass the last-level cache; FP32 form on large grids).
//
// Two arithmetic forms share the templates:
//   R = double, DEV = false: FP64 values as defined by the paper;
//   R = float,  DEV = true : FP32 deviations f - w p0, g_{1..8},
//     hbar_{0..8} - w rho cv Tr (and FP64 g_0), with
//     the linear reference Tr = Ts + Tg y taken at the row of the stored
//     value (a population moving to the next row changes reference by
//     w rho cv Tg xi_y);
//     Delta p and Delta T come from them, and every equilibrium is written as
//     a deviation (w Delta p + rho cs^2 G, rho cv (Delta T w + T G), with
//     G = Gamma_i(u) - w_i), so no large value is formed and then subtracted.
#pragma once

#include "host_layout.h"
#include "lattice.h"

namespace lbe {

// plane of distribution q (0..26 = f, g, hbar; not 9 or 18, the rest planes)
__host__ __device__ constexpr int plane_of(int q) { return q < 9 ? q : (q < 18 ? q - 1 : q - 2); }

// A rest population as stored (raw), and its value.  Rows loaded ahead keep
// the raw word in registers: converting at the load would make the wave wait
// for the load there, long before the row is used (measured: 20% slower).
template <int F> struct RestRaw { using T = double; };
template <> struct RestRaw<kRestF32> { using T = float; };
template <int F>
__device__ __forceinline__ double rest_decode(typename RestRaw<F>::T v) {
  return double(v);
}

// Addresses in the row-interleaved state (host_layout.h): the value of
// storage plane p at (x, y) sits at byte y * row_bytes + p * nx * sizeof(S)
// + x * sizeof(S).  Buffer accesses take the row's offset plus the lane's
// column as the per-lane offset and the plane's offset within the row as the
// scalar base.

// rest population of a site through the state's buffer descriptor (row_off:
// the row's byte offset, base: the rest plane's offset within a row)
template <typename S, int W>
__device__ __forceinline__ typename RestRaw<rest_fmt<S>(W)>::T rest_load_raw(
    __amdgpu_buffer_rsrc_t r, uint32_t row_off, int x, uint32_t base) {
  using T = typename RestRaw<rest_fmt<S>(W)>::T;
  return buf_load<T>(r, row_off + (uint32_t)x * (uint32_t)sizeof(T), base);
}
template <typename S, int W>
__device__ __forceinline__ double rest_load(__amdgpu_buffer_rsrc_t r, uint32_t row_off, int x,
                                            uint32_t base) {
  return rest_decode<rest_fmt<S>(W)>(rest_load_raw<S, W>(r, row_off, x, base));
}
template <typename S, int W, bool STREAM>
__device__ __forceinline__ void rest_store(double v, __amdgpu_buffer_rsrc_t r, uint32_t row_off,
                                           int x, uint32_t base) {
  using T = typename RestRaw<rest_fmt<S>(W)>::T;
  const uint32_t off = row_off + (uint32_t)x * (uint32_t)sizeof(T);
  if constexpr (STREAM) buf_store_stream<T>(T(v), r, off, base);
  else buf_store<T>(T(v), r, off, base);
}
// the same through plain pointers (set-up and conversion kernels): storage
// plane p of site (x, y) as an index into the state viewed as S[], and the
// rest populations
template <typename S>
__host__ __device__ __forceinline__ size_t plane_index(int p, size_t nx, size_t y, size_t x) {
  return y * (row_bytes<S>(nx) / sizeof(S)) + (size_t)p * nx + x;
}
template <typename S, int W>
__device__ __forceinline__ double rest_get(const void *state, size_t nx, size_t y, size_t x) {
  using T = typename RestRaw<rest_fmt<S>(W)>::T;
  return double(reinterpret_cast<const T *>(static_cast<const char *>(state) +
                                            y * row_bytes<S>(nx) + rest_base<S>(W, nx))[x]);
}
template <typename S, int W>
__device__ __forceinline__ void rest_set(void *state, size_t nx, size_t y, size_t x, double v) {
  using T = typename RestRaw<rest_fmt<S>(W)>::T;
  reinterpret_cast<T *>(static_cast<char *>(state) + y * row_bytes<S>(nx) +
                        rest_base<S>(W, nx))[x] = T(v);
}

// constants in the kernel's arithmetic type
template <typename R>
struct Consts {
  R rho, inv_rho, rcv, tauf0, dtauf, tauT0, dtauT, wg, gam3, kcap, epsalpha;
  R sigma0, sigmaT, bfx, bfy;
  __device__ explicit Consts(const StepArgs &a)
      : rho(R(a.rho)), inv_rho(R(1.0 / a.rho)), rcv(R(a.rcv)), tauf0(R(a.tauf0)),
        dtauf(R(a.dtauf)), tauT0(R(a.tauT0)), dtauT(R(a.dtauT)), wg(R(a.omg_g)),
        gam3(R(a.gam3)), kcap(R(a.kcap)), epsalpha(R(a.epsalpha)), sigma0(R(a.sigma0)),
        sigmaT(R(a.sigmaT)), bfx(R(a.rho * a.ax)), bfy(R(a.rho * a.ay)) {}
};

// One row of a lane's column: v[q] for the 25 storage planes (v[9], v[18]
// unused) and the two rest populations as stored.
template <typename R>
struct RowVals {
  R v[27];
  typename RestRaw<rest_fmt<R>(0)>::T g0r;
  typename RestRaw<rest_fmt<R>(1)>::T h0r;
  __device__ __forceinline__ double g0() const { return rest_decode<rest_fmt<R>(0)>(g0r); }
  __device__ __forceinline__ double h0() const { return rest_decode<rest_fmt<R>(1)>(h0r); }
};

// Plane-major layout of a state held in LDS by the small-grid kernel: g_0
// (FP64), then hbar_0, then the 25 storage planes, each n values with the
// site index y nx + x; every plane stays aligned to its element size, and
// the lanes of a wave, holding consecutive sites, touch consecutive banks.
template <typename S>
__host__ __device__ constexpr size_t lds_rest_off(int which, size_t n) {
  return which == 0 ? 0 : n * 8;
}
template <typename S>
__host__ __device__ constexpr size_t lds_plane_off(int p, size_t n) {
  return n * (8 + rest_bytes<S>(1)) + (size_t)p * n * sizeof(S);
}

// Moments of a loaded site: c (FP64), T or Delta T (FP64), p or Delta p
// (sum f).  With two densities T = sum hbar / (rho(c) cv); in the FP32 form
// the stored hbar deviates from w rho cv Trow (rho of the c = 0 fluid), so
// Delta T = (sum of deviations - c drho cv Trow) / (rho(c) cv), Trow given
// as tref.
template <typename R, bool VR = false>
__device__ __forceinline__ void site_moments(const RowVals<R> &r, double inv_rcv, double *c,
                                             double *T, R *p, double rho = 0.0,
                                             double drho = 0.0, double cv = 0.0,
                                             double tref = 0.0) {
  R cs = 0, hs = 0, f = 0;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    f += r.v[q];
    if (q > 0) {
      cs += r.v[9 + q];
      hs += r.v[18 + q];
    }
  }
  *c = r.g0() + double(cs);
  if (VR)
    *T = (r.h0() + double(hs) - *c * drho * cv * tref) / ((rho + *c * drho) * cv);
  else
    *T = (r.h0() + double(hs)) * inv_rcv;
  *p = f;
}

// The collision, diagnostics and field output of site (x, j).  cS/cC/cN,
// tS.., pS.. point at the ring entries west of the site in rows j-1, j, j+1
// (index 0 west, 1 centre, 2 east).
// With LDSOUT the post-collision values go to a state in LDS (lds_dst) in
// the plane-major layout of lds_plane_off instead of to a.dst.
template <typename S, typename R, bool DEV, int MODE, bool LDSOUT = false>
__device__ __forceinline__ void site_update(const StepArgs &a, const Consts<R> &k, int j, int x,
                                            const double *cS, const double *cC, const double *cN,
                                            const R *tS, const R *tC, const R *tN, const R *pS,
                                            const R *pC, const R *pN, const RowVals<R> &cur,
                                            double *acc, char *lds_dst = nullptr) {
  constexpr bool VR = (MODE & kVarRho) != 0;
  const int nx = a.nx, ny = a.ny;
  const size_t n = (size_t)nx * (size_t)ny;
  // order parameter and its stencils in FP64
  const double cd = cC[1];
  double gcx_d, gcy_d, lap_d, mu_d, tHt = 0.0;
  {
    const double e = cC[2], w = cC[0], nn = cN[1], s = cS[1];
    const double ne = cN[2], nw = cN[0], sw = cS[0], se = cS[2];
    gcx_d = (e - w) * (1.0 / 3.0) + (ne + se - nw - sw) * (1.0 / 12.0);
    gcy_d = (nn - s) * (1.0 / 3.0) + (ne + nw - se - sw) * (1.0 / 12.0);
    const double dx2 = (e - cd) + (w - cd), dy2 = (nn - cd) + (s - cd);
    const double dd = (ne - cd) + (nw - cd) + (se - cd) + (sw - cd);
    lap_d = (2.0 / 3.0) * (dx2 + dy2) + (1.0 / 6.0) * dd;
    mu_d = a.beta2 * cd * (cd - 1.0) * (2.0 * cd - 1.0) - a.eps2 * lap_d;
    if (MODE & kCurv) {
      // Hessian of c on the same nine points (exact on quadratics) and the
      // second derivative along the unit tangent t = (-gy, gx)/|grad c|,
      // which equals |grad c| div n for n = grad c/|grad c|
      const double hxx = (2.0 / 3.0) * dx2 - (1.0 / 3.0) * dy2 + (1.0 / 6.0) * dd;
      const double hyy = (2.0 / 3.0) * dy2 - (1.0 / 3.0) * dx2 + (1.0 / 6.0) * dd;
      const double hxy = 0.25 * ((ne - nw) - (se - sw));
      const double gg = gcx_d * gcx_d + gcy_d * gcy_d;
      if (gg > 0.0)
        tHt = (gcy_d * gcy_d * hxx - 2.0 * gcx_d * gcy_d * hxy + gcx_d * gcx_d * hyy) / gg;
    }
  }
  const R c = R(cd);
  const R Tv = tC[1];   // T, or Delta T = T - Trow in the FP32 form
  const R pv = pC[1];   // p, or Delta p
  // FP32 form: temperatures are stored relative to the linear reference
  // Ts + Tg y; Trow is its value at this row's centre
  const double Trow = DEV ? a.Ts + a.Tg * (double(j) + 0.5) : 0.0;
  // Stencils of T and p, the force and the velocity are evaluated in FP64.
  // Near an interface they are small differences of larger terms (the
  // capillary force against the pressure gradient in Fbar = F - grad p, the
  // momentum against the half force in u), so in the FP32 form the
  // arithmetic, not the storage, would otherwise set the error.
  auto grad = [&](const R *Sr, const R *Cr, const R *Nr, double *gx, double *gy) {
    *gx = (double(Cr[2]) - double(Cr[0])) * (1.0 / 3.0) +
          (double(Nr[2]) + double(Sr[2]) - double(Nr[0]) - double(Sr[0])) * (1.0 / 12.0);
    *gy = (double(Nr[1]) - double(Sr[1])) * (1.0 / 3.0) +
          (double(Nr[2]) + double(Nr[0]) - double(Sr[2]) - double(Sr[0])) * (1.0 / 12.0);
  };
  double gTx, gTy, gpx, gpy;
  grad(tS, tC, tN, &gTx, &gTy);
  grad(pS, pC, pN, &gpx, &gpy);
  if (DEV) gTy += a.Tg;   // the stencil is exact on the linear reference
  double jxd = 0.0, jyd = 0.0;
#pragma unroll
  for (int q = 1; q < 9; ++q) {
    if (kEx[q] != 0) jxd += double(kEx[q]) * double(cur.v[q]);
    if (kEy[q] != 0) jyd += double(kEy[q]) * double(cur.v[q]);
  }
  if (MODE & kTape) {
    const size_t s = (size_t)j * nx + x;
    double *tc = static_cast<double *>(a.tape);
    R *tr = reinterpret_cast<R *>(tc + n);
    tc[s] = cd;
    tr[s] = Tv;
    tr[n + s] = pv;
    tr[2 * n + s] = R(jxd);
    tr[3 * n + s] = R(jyd);
  }
  // closures
  const double Tm = DEV ? double(Tv) + (Trow - a.Tref) : double(Tv) - a.Tref;   // T - Tref
  const double sigma = a.sigma0 - a.sigmaT * Tm;
  const double gsx = -a.sigmaT * gTx, gsy = -a.sigmaT * gTy;
  const double g2 = gcx_d * gcx_d + gcy_d * gcy_d;
  const double gds = gcx_d * gsx + gcy_d * gsy;
  // capillary part along grad c: kcap sigma mu (potential form) or
  // -sigma eps alpha |grad c| div n (curvature form)
  const double ks = (MODE & kCurv) ? -a.epsalpha * sigma * tHt : a.kcap * sigma * mu_d;
  // two densities: rho(c) = rho + c drho, grad rho = drho grad c
  const double rho_s = VR ? a.rho + cd * a.drho : a.rho;
  const double grx = VR ? a.drho * gcx_d : 0.0, gry = VR ? a.drho * gcy_d : 0.0;
  const double inv_rho = 1.0 / rho_s;
  const double Fxd = ks * gcx_d + a.epsalpha * (g2 * gsx - gds * gcx_d) + rho_s * a.ax;
  const double Fyd = ks * gcy_d + a.epsalpha * (g2 * gsy - gds * gcy_d) + rho_s * a.ay;
  const double uxd = 3.0 * jxd * inv_rho + 0.5 * Fxd * inv_rho;
  const double uyd = 3.0 * jyd * inv_rho + 0.5 * Fyd * inv_rho;
  if (MODE & kPress) {
    // the pressure of Eq. 9: p = sum f + (1/2) u.grad(rho cs^2)
    a.pc_out[(size_t)j * nx + x] = double(pv) + (0.5 / 3.0) * (uxd * grx + uyd * gry);
    return;
  }
  const R ux = R(uxd), uy = R(uyd);
  // F - grad p drives c (Eq. 12); F-bar = grad(rho cs^2) - grad p + F
  // drives hbar (Sec. III)
  const R Fbx = R(Fxd - gpx), Fby = R(Fyd - gpy);
  const R Fhx = VR ? R(Fxd - gpx + grx / 3.0) : Fbx, Fhy = VR ? R(Fyd - gpy + gry / 3.0) : Fby;

  if (MODE & kDiag) {
    const double Td = DEV ? double(Tv) + Trow : double(Tv);
    const double yy = double(j) + 0.5, xx = double(x) + 0.5;
    acc[0] += cd;
    acc[1] += (VR ? rho_s * a.cv : a.rcv) * Td;
    acc[2] += cd * yy;
    acc[3] += cd * xx;
    if (cd >= 0.5) {
      acc[4] += cd;
      acc[5] += cd * double(uy);
    }
    const double chk = cd + Td + double(pv) + double(ux) + double(uy);
    if (!isfinite(chk)) acc[6] += 1.0;
  }
  if (MODE & kFields) {
    const size_t s = (size_t)j * nx + x;
    if (a.phi) a.phi[s] = 2.0 * cd - 1.0;
    if (a.ux) a.ux[s] = double(ux);
    if (a.uy) a.uy[s] = double(uy);
    if (a.p) a.p[s] = DEV ? double(pv) + a.p0 : double(pv);
    if (a.T) a.T[s] = DEV ? double(Tv) + Trow : double(Tv);
  }
  if (MODE & kStore) {
    // one descriptor for the whole destination state (below 4 GiB); a
    // plane's segment within a row is selected by a scalar offset
    const __amdgpu_buffer_rsrc_t rd = plane_rsrc(a.dst, state_bytes_for<S>(n));
    const uint32_t pbytes = (uint32_t)(nx * sizeof(S));   // a plane's segment of a row
    const uint32_t RB = (uint32_t)row_bytes<S>(nx);
    const R ch = c < R(0) ? R(0) : (c > R(1) ? R(1) : c);
    const double wfd = 1.0 / (a.tauf0 + double(ch) * a.dtauf), cfd = 1.0 - 0.5 * wfd;
    const double usqd = uxd * uxd + uyd * uyd;
    const R wT = R(1) / (k.tauT0 + ch * k.dtauT);
    const R wg = k.wg;
    const R usq = ux * ux + uy * uy;
    // temperature in FP64 for the rest population, in R for the others
    double hs = 0.0;
#pragma unroll
    for (int q = 1; q < 9; ++q) hs += double(cur.v[18 + q]);
    const double rcv_s = VR ? rho_s * a.cv : a.rcv;
    // two densities, FP32 form: the deviations are taken from w rho cv Trow
    // with the density of the c = 0 fluid; hoff = (rho(c) - rho) cv Trow
    const double hoff_d = (VR && DEV) ? cd * a.drho * a.cv * Trow : 0.0;
    const double Td = (cur.h0() + hs - hoff_d) / rcv_s;   // T or Delta T, FP64
    const double Tfull_d = DEV ? Td + Trow : Td;
    const R Tfull = R(Tfull_d);
    const R rcvT = (VR ? R(rcv_s) : k.rcv) * Tfull;
    const R gmu = R(a.gam3 * mu_d);
    const R cgf = R(1) - R(0.5) * wg, chf = R(1) - R(0.5) * wT;
    const R irho = VR ? R(inv_rho) : k.inv_rho;
    const R src_g = R(3) * c * irho;          // c / (rho cs^2)
    const R src_h = R(3) * irho;              // 1 / (rho cs^2)
    const bool walls = a.walls_y != 0;
    const bool bot = walls && j == 0, top = walls && j == ny - 1;
    const uint32_t own = (uint32_t)j * RB;   // this row's offset
    // value of plane q to site (xs, row) (row_off = row * RB)
    auto st = [&](int q, int row, uint32_t row_off, int xs, R val) {
      if constexpr (LDSOUT)
        *reinterpret_cast<S *>(lds_dst + lds_plane_off<S>(plane_of(q), n) +
                               ((size_t)row * nx + xs) * sizeof(S)) = S(val);
      else
        buf_store<S>(S(val), rd, row_off + (uint32_t)xs * (uint32_t)sizeof(S),
                     (uint32_t)plane_of(q) * pbytes);
    };
    // stores whose lines this wave writes whole
    constexpr bool stream = (MODE & kStream) != 0;
    auto st_whole = [&](int q, int row, uint32_t row_off, int xs, R val) {
      const uint32_t off = row_off + (uint32_t)xs * (uint32_t)sizeof(S);
      if constexpr (LDSOUT)
        *reinterpret_cast<S *>(lds_dst + lds_plane_off<S>(plane_of(q), n) +
                               ((size_t)row * nx + xs) * sizeof(S)) = S(val);
      else if constexpr (stream)
        buf_store_stream<S>(S(val), rd, off, (uint32_t)plane_of(q) * pbytes);
      else
        buf_store<S>(S(val), rd, off, (uint32_t)plane_of(q) * pbytes);
    };
    // FP32 form: what the eight moving populations of g and hbar give away in
    // this collision, as stored (sum of old - new, each difference of two
    // nearby FP32 values)
    R dg = 0, dh = 0;
    R gsrc0 = 0, hsrc0 = 0, G0 = 0, gam0 = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const R w = wq<R>(i);
      const R e = R(kEx[i]) * ux + R(kEy[i]) * uy;
      const R G = w * (R(3) * e + R(4.5) * e * e - R(1.5) * usq);  // Gamma_i - w_i
      const R gam = w + G;
      const R cxu = R(kEx[i]) - ux, cyu = R(kEy[i]) - uy;
      const R fbe = Fbx * cxu + Fby * cyu;
      const R fhe = VR ? Fhx * cxu + Fhy * cyu : fbe;
      // f (Eqs. 6-7): f^eq = w p + rho cs^2 G, in FP64.  Near an interface
      // the forcing term carries the capillary force, which the pressure
      // gradient balances; FP32 weights and Gamma_i would leave a relative
      // bias of ~1e-8 in that balance, a spurious force whose viscous
      // response grows over R^2 / nu steps.
      const double wd = wq<double>(i);
      const double ed = double(kEx[i]) * uxd + double(kEy[i]) * uyd;
      const double Gd = wd * (3.0 * ed + 4.5 * ed * ed - 1.5 * usqd);
      const double fed = Fxd * (double(kEx[i]) - uxd) + Fyd * (double(kEy[i]) - uyd);
      const double feqd = wd * double(pv) + rho_s * (1.0 / 3.0) * Gd;
      const double vd = double(cur.v[i]);
      // with two densities the forcing adds (xi - u).grad(rho cs^2)
      // (Gamma_i(u) - Gamma_i(0)) (Eq. 6); Gamma_i(0) = w_i
      const double srcf = VR ? fed * (wd + Gd) +
                                   (1.0 / 3.0) * (grx * (double(kEx[i]) - uxd) +
                                                  gry * (double(kEy[i]) - uyd)) * Gd
                             : fed * (wd + Gd);
      const R fo = R(vd - wfd * (vd - feqd) + cfd * srcf);
      // g (Eqs. 12-14): g^eq_0 = c - (1 - w0) 3 Gamma mu + c G_0,
      //                 g^eq_i = w_i 3 Gamma mu + c G_i
      const R gsrc = cgf * src_g * fbe * gam;
      // hbar (Eqs. 22, 25): h^eq = rho cv T Gamma_i
      const R heq_full = rcvT * gam;
      const R hsrc = chf * src_h * fhe * heq_full;
      if (i == 0) {
        st_whole(0, j, own, x, fo);
        gsrc0 = gsrc;
        hsrc0 = hsrc;
        G0 = G;
        gam0 = gam;
        continue;
      }
      const R geq = w * gmu + c * G;
      const R go = cur.v[9 + i] - wg * (cur.v[9 + i] - geq) + gsrc;
      R heq;
      if constexpr (DEV && VR)
        heq = R(rcv_s) * (Tv * w + Tfull * G) + w * R(hoff_d);
      else
        heq = DEV ? k.rcv * (Tv * w + Tfull * G) : heq_full;
      const R ho = cur.v[18 + i] - wT * (cur.v[18 + i] - heq) + hsrc;
      dg += cur.v[9 + i] - go;
      // push to x + xi_i
      const bool out = (kEy[i] < 0 && bot) || (kEy[i] > 0 && top);
      if (out) {
        // reflected into the opposite direction at this site
        const int o = kOpp[i];
        const double *tw = kEy[i] < 0 ? a.twb : a.twt;
        const R twv = DEV ? R(tw[x] - Trow) : R(tw[x]);
        st(o, j, own, x, fo);
        st(9 + o, j, own, x, go);
        if constexpr (DEV && VR)
          st(18 + o, j, own, x, R(2) * w * (R(rcv_s) * twv + R(hoff_d)) - ho);
        else
          st(18 + o, j, own, x, R(2) * w * (VR ? R(rcv_s) : k.rcv) * twv - ho);
        dh += cur.v[18 + i] - ho;
      } else {
        int xd = x + kEx[i];
        xd = xd < 0 ? xd + nx : (xd >= nx ? xd - nx : xd);
        int yd = j + kEy[i];
        yd = yd < 0 ? yd + ny : (yd >= ny ? yd - ny : yd);
        const uint32_t ro = (uint32_t)yd * RB;
        if (kEx[i] == 0) {
          st_whole(i, yd, ro, xd, fo);
          st_whole(9 + i, yd, ro, xd, go);
        } else {
          st(i, yd, ro, xd, fo);
          st(9 + i, yd, ro, xd, go);
        }
        // a move to the next row changes the reference by Tg xi_y
        const R shift = DEV && kEy[i] != 0 ? R(kEy[i]) * w * k.rcv * R(a.Tg) : R(0);
        const R hst = ho - shift;
        if (kEx[i] == 0)
          st_whole(18 + i, yd, ro, xd, hst);
        else
          st(18 + i, yd, ro, xd, hst);
        dh += (cur.v[18 + i] - hst) - shift;
      }
    }
    // rest populations, formed in FP64
    double gnew, hnew;
    if (DEV) {
      // The collision conserves c = sum g and rho cv T = sum hbar at the site,
      // so the rest populations receive exactly what the eight stored FP32
      // values gave away: the FP64 g_0 takes up their rounding, and c is
      // transported without a systematic drift; hbar_0 is then rounded once
      // to its FP32 deviation.
      gnew = cur.g0() + double(dg);
      hnew = cur.h0() + double(dh);
    } else {
      // Eqs. 12-14 as printed: g_0 - w_g (g_0 - g^eq_0) with
      // g^eq_0 = c - (1 - w0) 3 Gamma mu + c G_0 and c = sum g
      const double w0 = wq<double>(0);
      const double geq0 = cd - (1.0 - w0) * double(gmu) + cd * double(G0);
      gnew = cur.g0() - double(wg) * (cur.g0() - geq0) + double(gsrc0);
      const double hdiff = cur.h0() - rcv_s * Tfull_d * double(gam0);
      hnew = cur.h0() + double(-wT * R(hdiff) + hsrc0);
    }
    if constexpr (LDSOUT) {
      using T0 = typename RestRaw<rest_fmt<S>(0)>::T;
      using T1 = typename RestRaw<rest_fmt<S>(1)>::T;
      const size_t so = (size_t)j * nx + x;
      *reinterpret_cast<T0 *>(lds_dst + lds_rest_off<S>(0, n) + so * sizeof(T0)) = T0(gnew);
      *reinterpret_cast<T1 *>(lds_dst + lds_rest_off<S>(1, n) + so * sizeof(T1)) = T1(hnew);
    } else {
      rest_store<S, 0, stream>(gnew, rd, own, x, (uint32_t)rest_base<S>(0, nx));
      rest_store<S, 1, stream>(hnew, rd, own, x, (uint32_t)rest_base<S>(1, nx));
    }
  }
}

// deterministic block reduction of the per-lane diagnostic sums: fixed
// butterfly within each wave, then the wave partials summed in order
template <int NWAVES>
__device__ __forceinline__ void block_partials(const double *acc, double (*red)[kNumPartials],
                                               int lane, double *out) {
  const int wave = lane >> 6, wl = lane & 63;
#pragma unroll
  for (int q = 0; q < kNumPartials; ++q) {
    double v = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (wl == 0) red[wave][q] = v;
  }
  __syncthreads();
  if (lane < kNumPartials) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVES; ++w) s += red[w][lane];
    out[lane] = s;
  }
}

// Block barrier that waits for this wave's LDS operations only.  The ring
// is the only data shared within a block, so outstanding global loads (the
// rows prefetched for later iterations) need not be drained, as the
// compiler's barrier would do.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// ---------------------------------------------------------------------------
// Register-fed variant.
template <typename S, typename R, bool DEV, int MODE, int NW, int PIPE>
__global__ void __launch_bounds__(64 * NW)
step_kernel(const StepArgs a) {
  constexpr int BX = 64 * NW;
  __shared__ double ringc[4][BX + 2];     // c
  __shared__ R ringt[4][BX + 2];          // T (or Delta T)
  __shared__ R ringp[4][BX + 2];          // p (or Delta p)
  __shared__ double red[NW][kNumPartials];

  const int nx = a.nx, ny = a.ny;
  const bool walls = a.walls_y != 0;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int strip = t % a.nstrips;
  const int chunk = t / a.nstrips;
  const int x0 = strip * BX;
  const int nact = min(BX, nx - x0);
  const int lane = threadIdx.x;
  const bool act = lane < nact;
  const int x = x0 + lane;
  const int y0 = chunk * a.rows_per_chunk;
  const int y1 = min(y0 + a.rows_per_chunk, ny);
  const size_t n = (size_t)nx * (size_t)ny;
  const S *__restrict__ src = static_cast<const S *>(a.src);
  const Consts<R> k(a);
  const double inv_rcv = 1.0 / a.rcv;

  // helper lanes: 0..2 sum the left halo column's c, T, p, 3..5 the right
  // one's.  Eight-wave strips and the FP64 step spread them over the waves
  // (the last ceil(6 / NW) lanes of each), so that no wave carries all the
  // halo loads; measured on 4096^2: FP32 eight waves 1.1% faster, FP64 four
  // waves 1.3% faster, but the FP32 four-wave step on 4096 x 1024 0.4% slower, so
  // there lanes 0..5 of the last wave keep them
  constexpr bool kSpread = NW >= 6 || sizeof(S) == 8;
  constexpr int kHPW = (6 + NW - 1) / NW;   // helpers per wave
  const int hli = 63 - (lane & 63);
  const int hl = kSpread ? (hli < kHPW ? (lane >> 6) * kHPW + hli : -1) : lane - (BX - 64);
  const bool halo = hl >= 0 && hl < 6;
  const int hside = hl / 3;
  const int hfield = hl - 3 * hside;  // 0: c, 1: T, 2: p
  const int hx = hside == 0 ? (x0 == 0 ? nx - 1 : x0 - 1) : (x0 + nact == nx ? 0 : x0 + nact);
  const int hpos = hside == 0 ? 0 : nact + 1;

  // one descriptor for the whole source state (below 4 GiB); a plane's
  // segment within a row is selected by a scalar offset
  const __amdgpu_buffer_rsrc_t rsrc = plane_rsrc(src, state_bytes_for<S>(n));
  const uint32_t pbytes = (uint32_t)(nx * sizeof(S));   // a plane's segment of a row
  const uint32_t RB = (uint32_t)row_bytes<S>(nx);
  auto ld = [&](int q, uint32_t row_off, int xs) {
    return R(buf_load<S>(rsrc, row_off + (uint32_t)xs * (uint32_t)sizeof(S),
                         (uint32_t)plane_of(q) * pbytes));
  };
  const uint32_t rb0 = (uint32_t)rest_base<S>(0, nx), rb1 = (uint32_t)rest_base<S>(1, nx);
  auto ldd = [&](int which, uint32_t row_off, int xs) {
    return which == 0 ? rest_load<S, 0>(rsrc, row_off, xs, rb0)
                      : rest_load<S, 1>(rsrc, row_off, xs, rb1);
  };
  auto wrap_row = [&](int r) { return r < 0 ? r + ny : (r >= ny ? r - ny : r); };
  auto is_ghost = [&](int row) { return walls && (row < 0 || row >= ny); };

  auto load_row = [&](int row, RowVals<R> &r) {
    if (act) {
      const uint32_t ro = (uint32_t)row * RB;
#pragma unroll
      for (int q = 0; q < 27; ++q)
        if (q != 9 && q != 18) r.v[q] = ld(q, ro, x);
      r.g0r = rest_load_raw<S, 0>(rsrc, ro, x, rb0);
      r.h0r = rest_load_raw<S, 1>(rsrc, ro, x, rb1);
    }
  };
  // a helper lane's halo values: the nine planes of its field, and the FP64
  // rest population for c and T
  struct HaloVals {
    R v[9];
    typename RestRaw<rest_fmt<S>(0)>::T g0r;   // c helpers
    typename RestRaw<rest_fmt<S>(1)>::T h0r;   // T helpers
  };
  auto load_halo = [&](int row, HaloVals &h) {
    if (halo) {
      const uint32_t ro = (uint32_t)row * RB;
      if (hfield == 2) {
#pragma unroll
        for (int q = 0; q < 9; ++q) h.v[q] = ld(q, ro, hx);
      } else {
#pragma unroll
        for (int q = 1; q < 9; ++q) h.v[q] = ld(9 * (hfield + 1) + q, ro, hx);
        if (hfield == 0) h.g0r = rest_load_raw<S, 0>(rsrc, ro, hx, rb0);
        else h.h0r = rest_load_raw<S, 1>(rsrc, ro, hx, rb1);
      }
    }
  };
  // with two densities the ring's pressure is that of Eq. 9, computed by the
  // pressure pass of the same source state
  constexpr bool VR = (MODE & kVarRho) != 0;
  constexpr bool VRP = VR && !(MODE & kPress);
  // the FP32 form's temperature reference at the centre of a row
  auto tref_of = [&](int row) { return DEV ? a.Ts + a.Tg * (double(row) + 0.5) : 0.0; };
  auto put_own = [&](int slot, const RowVals<R> &r, int row) {
    if (act) {
      double c, T;
      R p;
      site_moments<R, VR>(r, inv_rcv, &c, &T, &p, a.rho, a.drho, a.cv, tref_of(row));
      ringc[slot][lane + 1] = c;
      ringt[slot][lane + 1] = R(T);
      ringp[slot][lane + 1] = VRP ? R(a.pc[(size_t)row * nx + x]) : p;
    }
  };
  // halo moments from prefetched values (PIPE 2)
  auto put_halo = [&](int slot, const HaloVals &h) {
    if (halo) {
      if (hfield == 0) {
        R cs = 0;
#pragma unroll
        for (int q = 1; q < 9; ++q) cs += h.v[q];
        ringc[slot][hpos] = rest_decode<rest_fmt<S>(0)>(h.g0r) + double(cs);
      } else if (hfield == 1) {
        R hs = 0;
#pragma unroll
        for (int q = 1; q < 9; ++q) hs += h.v[q];
        ringt[slot][hpos] = R((rest_decode<rest_fmt<S>(1)>(h.h0r) + double(hs)) * inv_rcv);
      } else {
        R f = 0;
#pragma unroll
        for (int q = 0; q < 9; ++q) f += h.v[q];
        ringp[slot][hpos] = f;
      }
    }
  };
  // halo moments loaded and summed in place (PIPE 0, 1)
  auto put_halo_direct = [&](int slot, int row) {
    if (halo) {
      const uint32_t ro = (uint32_t)row * RB;
      if (hfield == 0) {
        R cs = 0;
#pragma unroll
        for (int q = 1; q < 9; ++q) cs += ld(9 + q, ro, hx);
        ringc[slot][hpos] = ldd(0, ro, hx) + double(cs);
      } else if (hfield == 1) {
        R hs = 0;
#pragma unroll
        for (int q = 1; q < 9; ++q) hs += ld(18 + q, ro, hx);
        if (VR) {
          R cs = 0;
#pragma unroll
          for (int q = 1; q < 9; ++q) cs += ld(9 + q, ro, hx);
          const double ch = ldd(0, ro, hx) + double(cs);
          ringt[slot][hpos] =
              R((ldd(1, ro, hx) + double(hs) - ch * a.drho * a.cv * tref_of(row)) /
                ((a.rho + ch * a.drho) * a.cv));
        } else {
          ringt[slot][hpos] = R((ldd(1, ro, hx) + double(hs)) * inv_rcv);
        }
      } else if (VRP) {
        ringp[slot][hpos] = R(a.pc[(size_t)row * nx + hx]);
      } else {
        R f = 0;
#pragma unroll
        for (int q = 0; q < 9; ++q) f += ld(q, ro, hx);
        ringp[slot][hpos] = f;
      }
    }
  };
  // ghost row beyond a wall from the adjacent row's slot: c and p mirrored,
  // T_ghost = 2 T_wall - T (in deviations 2 (T_wall - Ts) - Delta T); each
  // lane reads only entries it wrote itself
  // (FP32 form: Delta T of the ghost row against the reference of its own
  // row, which is 2 (T_wall - Tref(wall)) - Delta T for a linear reference)
  auto put_ghost = [&](int slot, int from, const double *tw) {
    const double twref = DEV ? a.Ts + (tw == a.twb ? 0.0 : a.Tg * double(ny)) : 0.0;
    if (act) {
      ringc[slot][lane + 1] = ringc[from][lane + 1];
      ringp[slot][lane + 1] = ringp[from][lane + 1];
      const R twv = DEV ? R(tw[x] - twref) : R(tw[x]);
      ringt[slot][lane + 1] = R(2) * twv - ringt[from][lane + 1];
    }
    if (halo) {
      if (hfield == 0) {
        ringc[slot][hpos] = ringc[from][hpos];
      } else if (hfield == 1) {
        const R twv = DEV ? R(tw[hx] - twref) : R(tw[hx]);
        ringt[slot][hpos] = R(2) * twv - ringt[from][hpos];
      } else {
        ringp[slot][hpos] = ringp[from][hpos];
      }
    }
  };
  auto moments_or_ghost = [&](int row, int adj, RowVals<R> &tmp) {
    if (is_ghost(row)) {
      put_ghost(row & 3, adj & 3, row < 0 ? a.twb : a.twt);
    } else {
      load_row(wrap_row(row), tmp);
      put_own(row & 3, tmp, wrap_row(row));
      put_halo_direct(row & 3, wrap_row(row));
    }
  };

  double acc[kNumPartials];
#pragma unroll
  for (int q = 0; q < kNumPartials; ++q) acc[q] = 0.0;

  RowVals<R> cur, nxt, nxt2;
  HaloVals hnxt, hnxt2;
#pragma unroll
  for (int q = 0; q < 27; ++q) cur.v[q] = nxt.v[q] = R(0);
  cur.g0r = nxt.g0r = 0;
  cur.h0r = nxt.h0r = 0;
  load_row(y0, cur);
  put_own(y0 & 3, cur, y0);
  put_halo_direct(y0 & 3, y0);
  moments_or_ghost(y0 - 1, y0, nxt);
  if (PIPE == 2 && !is_ghost(y0 + 1)) {
    load_row(wrap_row(y0 + 1), nxt);
    load_halo(wrap_row(y0 + 1), hnxt);
  }
  for (int j = y0; j < y1; ++j) {
    if (PIPE == 2) {
      // issue the loads of row j + 2, then the moments of row j + 1 from the
      // values loaded one iteration earlier: a row's loads have a whole
      // collision to arrive, and the barrier waits for LDS only
      if (j + 2 <= y1 && !is_ghost(j + 2)) {
        load_row(wrap_row(j + 2), nxt2);
        load_halo(wrap_row(j + 2), hnxt2);
      }
      if (is_ghost(j + 1)) {
        put_ghost((j + 1) & 3, j & 3, a.twt);
      } else {
        put_own((j + 1) & 3, nxt, wrap_row(j + 1));
        put_halo((j + 1) & 3, hnxt);
      }
      lds_barrier();
    } else {
      // moments of row j + 1 (PIPE 1 keeps its values for the next collision)
      moments_or_ghost(j + 1, j, nxt);
      __syncthreads();
      if (PIPE == 0) load_row(j, cur);   // second read of row j, from cache
    }
    if (act) {
      const int l = lane;
      site_update<S, R, DEV, MODE>(a, k, j, x, &ringc[(j - 1) & 3][l], &ringc[j & 3][l],
                                   &ringc[(j + 1) & 3][l], &ringt[(j - 1) & 3][l],
                                   &ringt[j & 3][l], &ringt[(j + 1) & 3][l],
                                   &ringp[(j - 1) & 3][l], &ringp[j & 3][l],
                                   &ringp[(j + 1) & 3][l], cur, acc);
    }
    if (PIPE >= 1) cur = nxt;
    if (PIPE == 2) {
      nxt = nxt2;
      hnxt = hnxt2;
    }
  }
  if (MODE & kDiag)
    block_partials<NW>(acc, red, lane, a.partials + (size_t)blockIdx.x * kNumPartials);
  static_assert(!VR || PIPE == 1, "two densities: rows loaded one ahead");
}

// ---------------------------------------------------------------------------
// Small grids: many steps in one launch of one block.  A grid of a few
// thousand sites gives the per-step launch of step_kernel only a few
// hundred waves, and its step time is the latency of one pass (loads, LDS
// ring, collision, stores) plus the launch.  Here one block keeps the
// moments c, T, p of the whole grid in LDS (with a column of halo on each
// side and a ghost row beyond each wall), so a step is: every lane forms
// the moments of its sites, a barrier, every lane collides and pushes its
// sites into the other state (through L2: the two states of such a grid
// stay in cache), a barrier.  The site arithmetic is site_moments and
// site_update of the per-step kernel, and the halo and ghost values are
// formed exactly as its ring does, so the states are bitwise the same.
// One density; no diagnostics, fields or tape (the host runs the steps that
// need them through step_kernel).  All waves of a block share one CU and its
// L1, so the block barrier also orders the global stores of one step before
// the loads of the next.
// With RES both states also live in LDS, after the moments (16-byte
// aligned), plane-major (lds_plane_off): the source state is copied in at
// the start, every step reads and writes LDS only, and the last state is
// copied out to the global buffer that one launch per step would have left
// it in.  Blocks of at most kSmallMaxSites (512) lanes leave each lane twice
// the registers of a 1024-lane block, enough for the collision without
// spilling.
template <typename S, typename R, bool DEV, int MODE, bool RES>
__global__ void __launch_bounds__(kSmallMaxSites)
small_step_kernel(const StepArgs a0, void *other, int nsteps) {
  static_assert((MODE & (kDiag | kFields | kTape | kVarRho | kPress | kStream)) == 0,
                "small grids: plain steps only");
  extern __shared__ double smem[];
  const int nx = a0.nx, ny = a0.ny;
  const int W = nx + 2;                  // padded row: halo column on each side
  const int H = ny + 2;                  // ghost row beyond each wall (or wrap)
  double *lc = smem;                     // [H][W] c
  R *lt = reinterpret_cast<R *>(lc + (size_t)H * W);   // [H][W] T (or Delta T)
  R *lp = lt + (size_t)H * W;                          // [H][W] p (or Delta p)
  const bool walls = a0.walls_y != 0;
  const size_t n = (size_t)nx * (size_t)ny;
  const Consts<R> k(a0);
  const double inv_rcv = 1.0 / a0.rcv;
  const uint32_t pbytes = (uint32_t)(nx * sizeof(S));   // a plane's segment of a row
  const uint32_t RB = (uint32_t)row_bytes<S>(nx);
  const uint32_t rb0 = (uint32_t)rest_base<S>(0, nx), rb1 = (uint32_t)rest_base<S>(1, nx);
  const int nthr = blockDim.x;
  StepArgs a = a0;
  const void *srcp = a0.src;
  void *dstp = other;
  // resident states (RES): [2][state bytes] after the moments
  const size_t sbytes = state_bytes_for<S>(n);
  char *ls0 = reinterpret_cast<char *>(smem) + small_moment_bytes<R>(nx, ny);
  char *lsrc = ls0, *ldst = ls0 + sbytes;
  using T0 = typename RestRaw<rest_fmt<S>(0)>::T;
  using T1 = typename RestRaw<rest_fmt<S>(1)>::T;
  if constexpr (RES) {
    // row-interleaved global state -> plane-major LDS
    for (size_t i = threadIdx.x; i < n; i += nthr) {
      const size_t y = i / nx, x = i - y * nx;
      const char *g = static_cast<const char *>(a0.src) + y * RB;
#pragma unroll
      for (int p = 0; p < kNumS; ++p)
        reinterpret_cast<S *>(lsrc + lds_plane_off<S>(p, n))[i] =
            reinterpret_cast<const S *>(g + (size_t)p * pbytes)[x];
      reinterpret_cast<T0 *>(lsrc + lds_rest_off<S>(0, n))[i] =
          reinterpret_cast<const T0 *>(g + rb0)[x];
      reinterpret_cast<T1 *>(lsrc + lds_rest_off<S>(1, n))[i] =
          reinterpret_cast<const T1 *>(g + rb1)[x];
    }
    __syncthreads();
  }
  for (int step = 0; step < nsteps; ++step) {
    const __amdgpu_buffer_rsrc_t rsrc = plane_rsrc(srcp, state_bytes_for<S>(n));
    auto load_site = [&](int y, int x, RowVals<R> &r) {
      const uint32_t ro = (uint32_t)y * RB;
      if constexpr (RES) {
        const size_t i = (size_t)y * nx + x;
#pragma unroll
        for (int q = 0; q < 27; ++q)
          if (q != 9 && q != 18)
            r.v[q] = R(reinterpret_cast<const S *>(lsrc + lds_plane_off<S>(plane_of(q), n))[i]);
        r.g0r = reinterpret_cast<const T0 *>(lsrc + lds_rest_off<S>(0, n))[i];
        r.h0r = reinterpret_cast<const T1 *>(lsrc + lds_rest_off<S>(1, n))[i];
      } else {
#pragma unroll
        for (int q = 0; q < 27; ++q)
          if (q != 9 && q != 18)
            r.v[q] = R(buf_load<S>(rsrc, ro + (uint32_t)x * (uint32_t)sizeof(S),
                                   (uint32_t)plane_of(q) * pbytes));
        r.g0r = rest_load_raw<S, 0>(rsrc, ro, x, rb0);
        r.h0r = rest_load_raw<S, 1>(rsrc, ro, x, rb1);
      }
    };
    // moments of every site, with the halo columns and the ghost rows
    for (int s = threadIdx.x; s < (int)n; s += nthr) {
      const int x = s % nx, y = s / nx;
      RowVals<R> r;
      load_site(y, x, r);
      double c, T;
      R p;
      site_moments<R, false>(r, inv_rcv, &c, &T, &p);
      const R Tr = R(T);
      // this site's cell and its copies: the halo column across the x
      // wrap-around, and the row beyond a wall (a ghost) or across the
      // periodic y boundary
      const int rows[2] = {y + 1, y == 0 ? (walls ? 0 : ny + 1)
                                         : (y == ny - 1 ? (walls ? ny + 1 : 0) : -1)};
      const int cols[2] = {x + 1, x == 0 ? nx + 1 : (x == nx - 1 ? 0 : -1)};
      for (int iy = 0; iy < 2; ++iy) {
        if (rows[iy] < 0) continue;
        const bool ghost = iy == 1 && walls;
        for (int ix = 0; ix < 2; ++ix) {
          if (cols[ix] < 0) continue;
          const size_t cell = (size_t)rows[iy] * W + cols[ix];
          lc[cell] = c;
          lp[cell] = p;
          if (!ghost) {
            lt[cell] = Tr;
          } else {
            // beyond a wall: c and p mirrored, T_ghost = 2 T_wall - T with
            // the wall temperature of the cell's column (deviations against
            // the reference at the wall)
            const bool bot = rows[iy] == 0;
            const double *tw = bot ? a.twb : a.twt;
            const double twref = DEV ? a.Ts + (bot ? 0.0 : a.Tg * double(ny)) : 0.0;
            const int wc = cols[ix] == 0 ? nx - 1 : (cols[ix] == nx + 1 ? 0 : cols[ix] - 1);
            const R twv = DEV ? R(tw[wc] - twref) : R(tw[wc]);
            lt[cell] = R(2) * twv - Tr;
          }
        }
      }
    }
    __syncthreads();
    a.src = srcp;
    a.dst = dstp;
    double acc[kNumPartials];
    for (int s = threadIdx.x; s < (int)n; s += nthr) {
      const int x = s % nx, y = s / nx;
      RowVals<R> cur;
      load_site(y, x, cur);
      const size_t rS = (size_t)y * W + x, rC = rS + W, rN = rC + W;
      site_update<S, R, DEV, MODE, RES>(a, k, y, x, lc + rS, lc + rC, lc + rN, lt + rS,
                                        lt + rC, lt + rN, lp + rS, lp + rC, lp + rN, cur, acc,
                                        ldst);
    }
    __syncthreads();
    const void *t = srcp;
    srcp = dstp;
    dstp = const_cast<void *>(t);
    char *lt2 = lsrc;
    lsrc = ldst;
    ldst = lt2;
  }
  if constexpr (RES) {
    // the last state (plane-major LDS) to the buffer that holds it after an
    // alternation of nsteps steps (row-interleaved)
    for (size_t i = threadIdx.x; i < n; i += nthr) {
      const size_t y = i / nx, x = i - y * nx;
      char *g = static_cast<char *>(const_cast<void *>(srcp)) + y * RB;
#pragma unroll
      for (int p = 0; p < kNumS; ++p)
        reinterpret_cast<S *>(g + (size_t)p * pbytes)[x] =
            reinterpret_cast<const S *>(lsrc + lds_plane_off<S>(p, n))[i];
      reinterpret_cast<T0 *>(g + rb0)[x] = reinterpret_cast<const T0 *>(lsrc + lds_rest_off<S>(0, n))[i];
      reinterpret_cast<T1 *>(g + rb1)[x] = reinterpret_cast<const T1 *>(lsrc + lds_rest_off<S>(1, n))[i];
    }
  }
}

// ---------------------------------------------------------------------------
// Latency-bound grids: one plain step per launch in tiles of kTileX x kTileY
// sites, one site per lane.  The row-marching kernel gives such grids chunks
// of a row or two, and a chunk then waits for its own row, the rows above
// and below and their halo columns one after another.  Here every lane
// issues the loads of its own site and of at most one cell of the tile's
// one-site frame (or of the site that a frame cell beyond the grid copies)
// at once, forms the moments into an LDS tile, and after one barrier
// collides its site with site_update.  The tile's cells hold what the row
// kernel's ring holds (site_moments; beyond a wall c and p mirrored and
// 2 T_wall - T; periodic wrap otherwise), so the states are bitwise the same.
// Every mode of step_kernel but the streaming-store policy (diagnostics: one
// FP64 partial per block, as there); with two densities the pressure pass
// and the step, whose cells take p from the pressure plane as the ring does.
template <typename S, typename R, bool DEV, int MODE>
__global__ void __launch_bounds__(kTileX * kTileY)
tile_step_kernel(const StepArgs a) {
  static_assert((MODE & kStream) == 0, "tile kernel: default store policy");
  constexpr bool VR = (MODE & kVarRho) != 0;
  constexpr bool VRP = VR && !(MODE & kPress);
  constexpr int W = kTileX + 2, H = kTileY + 2;   // tile with its frame
  constexpr int kFrame = 2 * W + 2 * kTileY;      // cells of the frame
  constexpr int kWaves = kTileX * kTileY / 64;
  static_assert(kFrame <= kTileX * kTileY, "one frame cell per lane at most");
  __shared__ double lc[H * W];
  __shared__ R lt[H * W];
  __shared__ R lp[H * W];
  __shared__ double red[kWaves][kNumPartials];
  const int nx = a.nx, ny = a.ny;
  const bool walls = a.walls_y != 0;
  const size_t n = (size_t)nx * (size_t)ny;
  const Consts<R> k(a);
  const double inv_rcv = 1.0 / a.rcv;
  const int ntx = (nx + kTileX - 1) / kTileX;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % ntx) * kTileX, y0 = (tile / ntx) * kTileY;
  const int tid = threadIdx.x;
  const int lx = tid % kTileX, ly = tid / kTileX;
  const __amdgpu_buffer_rsrc_t rsrc = plane_rsrc(a.src, state_bytes_for<S>(n));
  const uint32_t pbytes = (uint32_t)(nx * sizeof(S));   // a plane's segment of a row
  const uint32_t RB = (uint32_t)row_bytes<S>(nx);
  const uint32_t rb0 = (uint32_t)rest_base<S>(0, nx), rb1 = (uint32_t)rest_base<S>(1, nx);
  auto load_site = [&](int y, int x, RowVals<R> &r) {
    const uint32_t ro = (uint32_t)y * RB;
#pragma unroll
    for (int q = 0; q < 27; ++q)
      if (q != 9 && q != 18)
        r.v[q] = R(buf_load<S>(rsrc, ro + (uint32_t)x * (uint32_t)sizeof(S),
                               (uint32_t)plane_of(q) * pbytes));
    r.g0r = rest_load_raw<S, 0>(rsrc, ro, x, rb0);
    r.h0r = rest_load_raw<S, 1>(rsrc, ro, x, rb1);
  };
  // a cell of the tile (cx, cy in 0..W-1, 0..H-1, frame included): the site
  // whose moments it holds, and whether it is a ghost beyond a wall (then the
  // moments of the wall row, transformed)
  struct Cell {
    int sx, sy, ghost;   // ghost: 0 none, -1 below the bottom wall, 1 above the top
  };
  auto cell_of = [&](int cx, int cy) {
    Cell c;
    int gx = x0 - 1 + cx, gy = y0 - 1 + cy;
    gx %= nx;
    c.sx = gx < 0 ? gx + nx : gx;
    c.ghost = 0;
    if (walls && gy < 0) {
      c.sy = 0;
      c.ghost = -1;
    } else if (walls && gy >= ny) {
      c.sy = ny - 1;
      c.ghost = 1;
    } else {
      gy %= ny;
      c.sy = gy < 0 ? gy + ny : gy;
    }
    return c;
  };
  auto put_cell = [&](int idx, const Cell &c, const RowVals<R> &r) {
    double cv, T;
    R p;
    // with two densities T needs the reference temperature of the site's row
    const double tref = DEV ? a.Ts + a.Tg * (double(c.sy) + 0.5) : 0.0;
    site_moments<R, VR>(r, inv_rcv, &cv, &T, &p, a.rho, a.drho, a.cv, tref);
    const R Tr = R(T);
    lc[idx] = cv;
    lp[idx] = VRP ? R(a.pc[(size_t)c.sy * nx + c.sx]) : p;
    if (c.ghost == 0) {
      lt[idx] = Tr;
    } else {
      // beyond a wall: T_ghost = 2 T_wall - T with the wall temperature of
      // the cell's column (deviations against the reference at the wall)
      const bool bot = c.ghost < 0;
      const double *tw = bot ? a.twb : a.twt;
      const double twref = DEV ? a.Ts + (bot ? 0.0 : a.Tg * double(ny)) : 0.0;
      const R twv = DEV ? R(tw[c.sx] - twref) : R(tw[c.sx]);
      lt[idx] = R(2) * twv - Tr;
    }
  };
  // this lane's own cell, and its frame cell (lanes 0 .. kFrame-1): frame
  // rows cy = 0 and H-1 (W cells each), then columns cx = 0 and W-1 of the
  // tile's rows
  const int ocx = lx + 1, ocy = ly + 1;
  const Cell own = cell_of(ocx, ocy);
  int fcx = 0, fcy = 0;
  if (tid < W) {
    fcx = tid;
    fcy = 0;
  } else if (tid < 2 * W) {
    fcx = tid - W;
    fcy = H - 1;
  } else if (tid < 2 * W + kTileY) {
    fcx = 0;
    fcy = tid - 2 * W + 1;
  } else {
    fcx = W - 1;
    fcy = tid - 2 * W - kTileY + 1;
  }
  const bool has_frame = tid < kFrame;
  const Cell fr = cell_of(fcx, fcy);
  RowVals<R> cur, fv;
  load_site(own.sy, own.sx, cur);
  if (has_frame) load_site(fr.sy, fr.sx, fv);
  put_cell(ocy * W + ocx, own, cur);
  if (has_frame) put_cell(fcy * W + fcx, fr, fv);
  __syncthreads();
  const int x = x0 + lx, y = y0 + ly;
  double acc[kNumPartials];
#pragma unroll
  for (int q = 0; q < kNumPartials; ++q) acc[q] = 0.0;
  // On grids two or four tiles wide whose last tile holds 1 to 8 columns,
  // the lanes beyond the last column collide the site their cells wrapped
  // to: the same cells and loaded values as the lane that owns it, so they
  // store the same values to the same addresses (and add nothing to the
  // diagnostic sums).  Left idle there, they cost up to 45% more per step
  // (200 x 100 FP32: 8.7 against 5.8 us); the collision ran that much slower
  // in waves with only those few lanes active.  Elsewhere the extra
  // collisions cost 1-3% (40 x 100, 160 x 300, FP64 130 x 100 and
  // 264 x 100), so there they idle.
  const int tail = nx % kTileX;
  const bool wrap = tail > 0 && tail <= 8 && (ntx == 2 || ntx == 4);
  if (y < ny && (x < nx || wrap)) {
    const int rS = ly * W + lx, rC = rS + W, rN = rC + W;
    site_update<S, R, DEV, MODE>(a, k, y, x < nx ? x : x % nx, lc + rS, lc + rC, lc + rN,
                                 lt + rS, lt + rC, lt + rN, lp + rS, lp + rC, lp + rN, cur, acc);
    if ((MODE & kDiag) && x >= nx) {
#pragma unroll
      for (int q = 0; q < kNumPartials; ++q) acc[q] = 0.0;
    }
  }
  if (MODE & kDiag)
    block_partials<kWaves>(acc, red, tid, a.partials + (size_t)blockIdx.x * kNumPartials);
}

}  // namespace lbe
