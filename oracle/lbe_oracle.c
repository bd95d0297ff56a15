/*
 * lbe_oracle.c -- plain, slow, FP64 CPU oracle of the CSF lattice Boltzmann
 * step for thermocapillary flow (Zheng, Zheng & Zhai, arXiv:1412.6238).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no source with the HIP library: its own
 * lattice tables, its own parameter derivations, its own passes.
 *
 * One time step is written as separate whole-grid passes, in the order the
 * method defines them:
 *   A  moments          c = sum g  (Eq. 15), rho cv T = sum hbar (Eq. 26),
 *                       p = sum f, rho cs^2 u from sum xi f (Eq. 9)
 *                       (with two densities, rho = rho(c) and p gains
 *                       (dt/2) u.grad(rho cs^2) once u is known, Eq. 9)
 *   B  stencils         grad c, lap c, grad T, grad p (the paper needs them
 *                       in Eqs. 4, 12, 16, 25 but does not give a scheme;
 *                       isotropic nine-point stencils are the reading used)
 *                       and the Hessian of c (curvature form of Eq. 4 only)
 *   C  closures         mu = mu0(c) - eps^2 lap c (Sec. II, Eq. 16),
 *                       sigma(T) (Eq. 5), CSF force (Eqs. 3-4, with its
 *                       capillary part in the potential or curvature form),
 *                       u (Eq. 9), relaxation rates (Eqs. 6, 12, 25)
 *   D  collide          f (Eqs. 6-8), g (Eqs. 12-14), hbar (Eqs. 22, 25)
 *   E  stream           periodic x; halfway bounce-back for f and g and
 *                       anti-bounce-back (Dirichlet T) for hbar at walls
 *                       (Sec. IV boundary conditions)
 * Readings of passages the paper leaves open are marked READING below.
 *
 * Windows.  The grid held here may be a window (x0, y0, wx, wy) of a larger
 * global domain (NX, NY).  A neighbour that falls outside the window and is
 * not a wall is unknown and reads as NaN, so every value whose dependence
 * cone leaves the window turns into NaN while the interior stays exact.  With
 * the full domain as window this is the ordinary periodic / walled grid.
 *
 * Built with -O2 -ffp-contract=off so that no fused multiply-add changes the
 * rounding of the plain expressions below.  OpenMP (optional) splits rows of
 * the per-site passes only; every site is computed by one thread in a fixed
 * order and the diagnostic sums run serially, so results do not depend on
 * the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- D2Q9 lattice (implied by the weights of Eqs. 7, 8, 13, 14) ----------- */
#define NQ 9
static const int OX[NQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int OY[NQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double OW[NQ] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                              1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OOPP[NQ] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double OCS2 = 1.0 / 3.0; /* lattice sound speed squared */

typedef struct {
  int32_t NX, NY;              /* global domain */
  int32_t x0, y0, wx, wy;      /* window held by this oracle */
  int32_t walls_y;             /* 1: halfway walls at y=0 and y=NY; 0: periodic */
  int32_t csf_form;            /* capillary force: 0 potential, 1 curvature   */
  double rho, cv;              /* uniform density, specific heat */
  double tau_f[2];             /* flow relaxation time at c=0 and c=1 */
  double tau_T[2];             /* thermal relaxation time (tau_h + 1/2) */
  double tau_g, mobility;      /* CH relaxation time, mobility M */
  double width, beta;          /* tanh width W, double-well coefficient */
  double sigma0, sigmaT, Tref; /* sigma = sigma0 - sigmaT (T - Tref) */
  double force[2];             /* body acceleration a */
  double p0;                   /* reference pressure of the initial state */
  double rho2;                 /* density of the c = 1 fluid (rho: c = 0) */
} orc_params;

/* Diagnostic record, one FP64 value each. */
enum {
  ORC_D_MASS = 0,   /* sum c                                   */
  ORC_D_ENERGY,     /* sum rho cv T                            */
  ORC_D_SUM_CY,     /* sum c y  (y = j + 1/2)                  */
  ORC_D_SUM_CX,     /* sum c x  (x = i + 1/2)                  */
  ORC_D_MASS_THR,   /* sum c over sites with c >= 1/2          */
  ORC_D_CUY_THR,    /* sum c u_y over sites with c >= 1/2      */
  ORC_D_NONFINITE,  /* number of sites with a non-finite value */
  ORC_D_N
};

typedef struct orc {
  orc_params P;
  /* derived constants */
  double eps, alpha, kcap, Gam;
  int n;            /* wx * wy */
  double *F;        /* [27][n] current pre-collision state: f 0-8, g 9-17, h 18-26 */
  double *Fp;       /* [27][n] post-collision scratch */
  double *Twb, *Twt;/* [NX] wall temperatures, global columns */
  int *nb_kind;     /* [9][n] kind of the neighbour x + xi_k (k = 0 unused) */
  int *nb_loc;      /* [9][n] its local index, or of its mirror image       */
  int *nb_col;      /* [9][n] its global column                             */
  /* macroscopic scratch fields, [n] each */
  double *c, *T, *p, *jx, *jy;
  double *gcx, *gcy, *lapc, *gTx, *gTy, *gpx, *gpy;
  double *mu, *Fx, *Fy, *ux, *uy;
  double *hxx, *hxy, *hyy;   /* Hessian of c */
} orc;

/* ---- neighbour lookup ------------------------------------------------------
 * Kinds of neighbour of local site (i,j) at offset (dx,dy). */
enum { NB_IN = 0, NB_WALL_BOT = 1, NB_WALL_TOP = 2, NB_UNKNOWN = 3 };

static int wrapi(int a, int m) {
  int r = a % m;
  return r < 0 ? r + m : r;
}

/* Returns the kind; *loc receives the local index of the neighbour (NB_IN) or
 * of its mirror image across the wall (wall kinds, -1 if that image is
 * outside the window); *gcol receives the neighbour's global column. */
static int neighbour(const orc *o, int i, int j, int dx, int dy, int *loc,
                     int *gcol) {
  const orc_params *P = &o->P;
  int gx = wrapi(P->x0 + i + dx, P->NX);
  int li = wrapi(gx - P->x0, P->NX);
  *gcol = gx;
  int gy = P->y0 + j + dy;
  int kind = NB_IN;
  if (P->walls_y) {
    if (gy < 0) {
      kind = NB_WALL_BOT;
      gy = -1 - gy; /* mirror of row -1 is row 0 */
    } else if (gy >= P->NY) {
      kind = NB_WALL_TOP;
      gy = 2 * P->NY - 1 - gy;
    }
  } else {
    gy = wrapi(gy, P->NY);
  }
  int lj = P->walls_y ? gy - P->y0 : wrapi(gy - P->y0, P->NY);
  int inside = (li < P->wx) && (lj >= 0) && (lj < P->wy);
  *loc = inside ? lj * P->wx + li : -1;
  if (kind == NB_IN && !inside) return NB_UNKNOWN;
  return kind;
}

/* READING: the density of the mixture is linear in the order parameter,
 * rho(c) = rho1 + c (rho2 - rho1), unclamped so that grad rho = (rho2 - rho1)
 * grad c exactly.  The paper carries the density terms of Eqs. 6, 9 and the
 * F-bar of Sec. III but never states the closure rho(c). */
static double rho_of(const orc_params *P, double c) {
  return P->rho + c * (P->rho2 - P->rho);
}

/* Order of the sums over lattice directions in the moments and stencils:
 * index order; a build with -DORC_REVERSED_SUMS sums in reverse order, the
 * same arithmetic rounded differently, which the tests use only to measure
 * how far two correct FP64 evaluations of an ill-conditioned case drift
 * apart.  DIR(t, first) is the t-th direction of a loop starting at first. */
#ifdef ORC_REVERSED_SUMS
#define DIR(t, first) (NQ - 1 - (t) + (first))
#else
#define DIR(t, first) (t)
#endif

/* ---- pass A: moments of the pre-collision state --------------------------- */
static void pass_moments(orc *o) {
  const int n = o->n;
#pragma omp parallel for schedule(static)
  for (int s = 0; s < n; ++s) {
    double sf = 0.0, sg = 0.0, sh = 0.0, sx = 0.0, sy = 0.0;
    for (int t = 0; t < NQ; ++t) {
      const int k = DIR(t, 0);
      double fk = o->F[k * n + s];
      sf += fk;
      sx += OX[k] * fk;
      sy += OY[k] * fk;
      sg += o->F[(NQ + k) * n + s];
      sh += o->F[(2 * NQ + k) * n + s];
    }
    o->p[s] = sf;        /* Eq. 9 without its u.grad(rho cs^2) term (pass C2) */
    o->jx[s] = sx;
    o->jy[s] = sy;
    o->c[s] = sg;        /* Eq. 15 */
    o->T[s] = sh / (rho_of(&o->P, sg) * o->P.cv);  /* Eq. 26 */
  }
}

/* ---- pass B: isotropic nine-point stencils ----------------------------------
 * READING: grad phi = (1/cs^2) sum_k w_k xi_k phi(x + xi_k) and
 * lap phi = (2/cs^2) sum_k w_k (phi(x + xi_k) - phi(x)).  Beyond a wall the
 * ghost values of c and p mirror the adjacent row (no flux of c, neutral
 * wetting) and the ghost temperature is 2 T_wall - T(adjacent), so that the
 * wall temperature holds halfway between. */
static void stencil_site(const orc *o, const double *c, const double *T,
                         const double *p, int i, int j, double out[10]) {
  const int s = j * o->P.wx + i;
  double gcx = 0, gcy = 0, lap = 0, gtx = 0, gty = 0, gpx = 0, gpy = 0;
  double hxx = 0, hxy = 0, hyy = 0;
  for (int t = 1; t < NQ; ++t) {
    const int k = DIR(t, 1);
    const int kind = o->nb_kind[k * o->n + s];
    const int loc = o->nb_loc[k * o->n + s];
    const int gcol = o->nb_col[k * o->n + s];
    double ck, tk, pk;
    if (kind == NB_UNKNOWN || loc < 0) {
      ck = tk = pk = NAN;
    } else if (kind == NB_IN) {
      ck = c[loc];
      tk = T ? T[loc] : 0.0;
      pk = p ? p[loc] : 0.0;
    } else {
      const double tw = (kind == NB_WALL_BOT) ? o->Twb[gcol] : o->Twt[gcol];
      ck = c[loc];
      pk = p ? p[loc] : 0.0;
      tk = T ? 2.0 * tw - T[loc] : 0.0;
    }
    const double w3 = OW[k] / OCS2;
    gcx += w3 * OX[k] * ck;
    gcy += w3 * OY[k] * ck;
    gtx += w3 * OX[k] * tk;
    gty += w3 * OY[k] * tk;
    gpx += w3 * OX[k] * pk;
    gpy += w3 * OY[k] * pk;
    lap += 2.0 * w3 * (ck - c[s]);
    /* Hessian from the fourth-order lattice moment: sum w xi_a xi_b (c_k - c)
     * = cs^4 (2 H_ab + delta_ab tr H) / 2 + O(dx^4), with cs^4 = 1/9 */
    hxx += OW[k] * (9.0 * OX[k] * OX[k] - 3.0) * (ck - c[s]);
    hyy += OW[k] * (9.0 * OY[k] * OY[k] - 3.0) * (ck - c[s]);
    hxy += OW[k] * 9.0 * OX[k] * OY[k] * ck;
  }
  out[0] = gcx; out[1] = gcy; out[2] = lap;
  out[3] = gtx; out[4] = gty; out[5] = gpx; out[6] = gpy;
  out[7] = hxx; out[8] = hxy; out[9] = hyy;
}

static void pass_stencils(orc *o) {
#pragma omp parallel for schedule(static)
  for (int j = 0; j < o->P.wy; ++j)
    for (int i = 0; i < o->P.wx; ++i) {
      double st[10];
      const int s = j * o->P.wx + i;
      stencil_site(o, o->c, o->T, o->p, i, j, st);
      o->gcx[s] = st[0]; o->gcy[s] = st[1]; o->lapc[s] = st[2];
      o->gTx[s] = st[3]; o->gTy[s] = st[4];
      o->gpx[s] = st[5]; o->gpy[s] = st[6];
      o->hxx[s] = st[7]; o->hxy[s] = st[8]; o->hyy[s] = st[9];
    }
}

/* ---- pass C: chemical potential, CSF force, velocity ----------------------- */
typedef struct {
  double mu, sigma, Fx, Fy, ux, uy, wf, wT, wg;
  double rho, grx, gry;  /* rho(c) and grad rho */
  double Fgx, Fgy;       /* F - grad p, the force term of the g equation (Eq. 12) */
  double Fbx, Fby;       /* F-bar = grad(rho cs^2) - grad p + F (Sec. III) */
} closure_t;

/* mu0 = dE0/dc for E0 = beta c^2 (c-1)^2 (Sec. II, c1 = 0, c2 = 1). */
static double mu_bulk(double beta, double c) {
  return 2.0 * beta * c * (c - 1.0) * (2.0 * c - 1.0);
}

static void closure_site(const orc *o, double c, double T, double jx, double jy,
                         double gcx, double gcy, double lapc, double gTx,
                         double gTy, double gpx, double gpy, double hxx,
                         double hxy, double hyy, closure_t *r) {
  const orc_params *P = &o->P;
  const double rho = rho_of(P, c);
  r->rho = rho;
  r->grx = (P->rho2 - P->rho) * gcx;
  r->gry = (P->rho2 - P->rho) * gcy;
  /* chemical potential, Sec. II below Eq. 16 */
  r->mu = mu_bulk(P->beta, c) - o->eps * o->eps * lapc;
  /* linear surface tension, Eq. 5; READING: sigmaT here is -sigma_T */
  r->sigma = P->sigma0 - P->sigmaT * (T - P->Tref);
  const double gsx = -P->sigmaT * gTx, gsy = -P->sigmaT * gTy;
  /* CSF force, Eqs. 3-4.  The tangential (Marangoni) part is grad_s(sigma)
   * delta with delta = eps alpha |grad c|^2.  The normal (capillary) part,
   * -sigma kappa n delta with n = grad c / |grad c| and kappa = div n, is
   * taken in one of two forms:
   *   0  READING: the potential form kcap sigma mu grad c, which follows
   *      from the stress form on the equilibrium profile;
   *   1  the curvature form as printed.  In two dimensions
   *      |grad c| div n = t.H.t with t the unit tangent and H the Hessian
   *      of c, so the force is -sigma eps alpha (t.H.t) grad c; where
   *      grad c vanishes the force does too. */
  const double g2 = gcx * gcx + gcy * gcy;
  const double gdots = gcx * gsx + gcy * gsy;
  const double ea = o->eps * o->alpha;
  double capx, capy;
  if (P->csf_form == 1) {
    const double tHt =
        g2 > 0.0 ? (gcy * gcy * hxx - 2.0 * gcx * gcy * hxy + gcx * gcx * hyy) / g2 : 0.0;
    capx = -r->sigma * ea * tHt * gcx;
    capy = -r->sigma * ea * tHt * gcy;
  } else {
    capx = o->kcap * r->sigma * r->mu * gcx;
    capy = o->kcap * r->sigma * r->mu * gcy;
  }
  r->Fx = capx + ea * (g2 * gsx - gdots * gcx) + rho * P->force[0];
  r->Fy = capy + ea * (g2 * gsy - gdots * gcy) + rho * P->force[1];
  /* Eq. 9.  READING: the half-force enters as (dt/2) cs^2 F, the first moment
   * of the forcing term of Eq. 6, so u = (sum xi f)/(rho cs^2) + F/(2 rho). */
  r->ux = jx / (rho * OCS2) + r->Fx / (2.0 * rho);
  r->uy = jy / (rho * OCS2) + r->Fy / (2.0 * rho);
  /* READING: relaxation times vary linearly with the clamped order parameter.
   * (Comparisons written so that a NaN passes through unchanged.) */
  double ch = c < 0.0 ? 0.0 : (c > 1.0 ? 1.0 : c);
  const double tf = P->tau_f[0] + ch * (P->tau_f[1] - P->tau_f[0]);
  const double tT = P->tau_T[0] + ch * (P->tau_T[1] - P->tau_T[0]);
  r->wf = 1.0 / tf;
  r->wT = 1.0 / tT;       /* 2 dt / (2 tau_h + dt) with tau_T = tau_h + 1/2 */
  r->wg = 1.0 / P->tau_g;
  /* F - grad p drives c (Eq. 12); F-bar = grad(rho cs^2) - grad p + F drives
   * hbar (Sec. III); they differ by the density gradient */
  r->Fgx = r->Fx - gpx;
  r->Fgy = r->Fy - gpy;
  r->Fbx = r->Fgx + OCS2 * r->grx;
  r->Fby = r->Fgy + OCS2 * r->gry;
}

static void pass_closures(orc *o) {
#pragma omp parallel for schedule(static)
  for (int s = 0; s < o->n; ++s) {
    closure_t r;
    closure_site(o, o->c[s], o->T[s], o->jx[s], o->jy[s], o->gcx[s], o->gcy[s],
                 o->lapc[s], o->gTx[s], o->gTy[s], o->gpx[s], o->gpy[s],
                 o->hxx[s], o->hxy[s], o->hyy[s], &r);
    o->mu[s] = r.mu;
    o->Fx[s] = r.Fx;
    o->Fy[s] = r.Fy;
    o->ux[s] = r.ux;
    o->uy[s] = r.uy;
  }
}

/* ---- pass C2: the pressure of Eq. 9 with two densities ----------------------
 * p = sum f + (dt/2) u.grad(rho cs^2), then the stencils again so that grad p
 * is taken of this p.  With one density the term is zero and the pass is
 * skipped. */
static void pass_pressure(orc *o) {
  const orc_params *P = &o->P;
  if (P->rho2 == P->rho) return;
  const double dr = P->rho2 - P->rho;
#pragma omp parallel for schedule(static)
  for (int s = 0; s < o->n; ++s)
    o->p[s] += 0.5 * OCS2 * dr * (o->ux[s] * o->gcx[s] + o->uy[s] * o->gcy[s]);
  pass_stencils(o);
}

/* ---- pass D: the three collisions at one site --------------------------------
 * in/out hold 27 values (f, g, hbar).  gamma_i(u) is Eq. 8. */
static void collide_site(const orc *o, const double *in, double c, double T,
                         double p, const closure_t *r, double *out) {
  const orc_params *P = &o->P;
  const double ux = r->ux, uy = r->uy;
  const double usq = ux * ux + uy * uy;
  const double rho = r->rho;
  for (int k = 0; k < NQ; ++k) {
    const double e = OX[k] * ux + OY[k] * uy;
    const double gam =
        OW[k] * (1.0 + e / OCS2 + 0.5 * ((e / OCS2) * (e / OCS2) - usq / OCS2));
    const double cxu = OX[k] - ux, cyu = OY[k] - uy;
    /* flow, Eqs. 6 and 7 */
    const double feq =
        OW[k] * (p + rho * OCS2 *
                         (e / OCS2 + 0.5 * ((e / OCS2) * (e / OCS2) - usq / OCS2)));
    /* F.(xi - u) Gamma_i(u) + (xi - u).grad(rho cs^2) (Gamma_i(u) - Gamma_i(0)),
     * with Gamma_i(0) = w_i */
    const double Sf = (r->Fx * cxu + r->Fy * cyu) * gam +
                      OCS2 * (r->grx * cxu + r->gry * cyu) * (gam - OW[k]);
    out[k] = in[k] - r->wf * (in[k] - feq) + (1.0 - 0.5 * r->wf) * Sf;
    /* order parameter, Eqs. 12-14 (w0 is the rest weight) */
    const double H = (k == 0)
                         ? (c - (1.0 - OW[0]) * o->Gam * r->mu / OCS2) / OW[0]
                         : o->Gam * r->mu / OCS2;
    const double geq =
        OW[k] * (H + c * (e / OCS2 + 0.5 * ((e / OCS2) * (e / OCS2) - usq / OCS2)));
    const double Sg = c * (cxu * r->Fgx + cyu * r->Fgy) / (rho * OCS2) * gam;
    out[NQ + k] = in[NQ + k] - r->wg * (in[NQ + k] - geq) + (1.0 - 0.5 * r->wg) * Sg;
    /* temperature, Eqs. 22 and 25 */
    const double heq = rho * P->cv * T * gam;
    const double Sh = (r->Fbx * cxu + r->Fby * cyu) / (rho * OCS2) * heq;
    out[2 * NQ + k] =
        in[2 * NQ + k] - r->wT * (in[2 * NQ + k] - heq) + (1.0 - 0.5 * r->wT) * Sh;
  }
}

static void pass_collide(orc *o) {
  const int n = o->n;
#pragma omp parallel for schedule(static)
  for (int s = 0; s < n; ++s) {
    double in[3 * NQ], out[3 * NQ];
    for (int k = 0; k < 3 * NQ; ++k) in[k] = o->F[k * n + s];
    closure_t r;
    closure_site(o, o->c[s], o->T[s], o->jx[s], o->jy[s], o->gcx[s], o->gcy[s],
                 o->lapc[s], o->gTx[s], o->gTy[s], o->gpx[s], o->gpy[s],
                 o->hxx[s], o->hxy[s], o->hyy[s], &r);
    collide_site(o, in, o->c[s], o->T[s], o->p[s], &r, out);
    for (int k = 0; k < 3 * NQ; ++k) o->Fp[k * n + s] = out[k];
  }
}

/* ---- pass E: streaming with boundary rules -----------------------------------
 * Pull form: F_k(x) <- F*_k(x - xi_k).  If x - xi_k lies beyond a halfway wall
 * the population that left x towards the wall comes back reversed:
 * f_k, g_k <- f*_opp(k), g*_opp(k) (no slip, no flux of c) and
 * hbar_k <- -hbar*_opp(k) + 2 w_k rho cv T_wall (fixed wall temperature).
 * READING: T_wall of a diagonal link is the wall value of x's own column. */
static void pass_stream(orc *o) {
  const orc_params *P = &o->P;
  const int n = o->n;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < P->wy; ++j)
    for (int i = 0; i < P->wx; ++i) {
      const int s = j * P->wx + i;
      /* rho cv of the boundary node (its pre-collision c) */
      const double rcv = rho_of(P, o->c[s]) * P->cv;
      for (int k = 0; k < NQ; ++k) {
        /* the source x - xi_k is the neighbour in direction opp(k) */
        const int kind = k == 0 ? NB_IN : o->nb_kind[OOPP[k] * n + s];
        const int loc = k == 0 ? s : o->nb_loc[OOPP[k] * n + s];
        if (kind == NB_IN) {
          o->F[k * n + s] = o->Fp[k * n + loc];
          o->F[(NQ + k) * n + s] = o->Fp[(NQ + k) * n + loc];
          o->F[(2 * NQ + k) * n + s] = o->Fp[(2 * NQ + k) * n + loc];
        } else if (kind == NB_UNKNOWN) {
          o->F[k * n + s] = NAN;
          o->F[(NQ + k) * n + s] = NAN;
          o->F[(2 * NQ + k) * n + s] = NAN;
        } else {
          const int gx = wrapi(P->x0 + i, P->NX);
          const double tw = (kind == NB_WALL_BOT) ? o->Twb[gx] : o->Twt[gx];
          const int q = OOPP[k];
          o->F[k * n + s] = o->Fp[q * n + s];
          o->F[(NQ + k) * n + s] = o->Fp[(NQ + q) * n + s];
          o->F[(2 * NQ + k) * n + s] =
              -o->Fp[(2 * NQ + q) * n + s] + 2.0 * OW[k] * rcv * tw;
        }
      }
    }
}

/* ---- public API ------------------------------------------------------------ */
#define OAPI __attribute__((visibility("default")))

static void derive(orc *o) {
  const orc_params *P = &o->P;
  /* READING: W is the tanh denominator of the planar profile (Sec. II),
   * W = eps sqrt(2/beta), and alpha normalises eps alpha int c'^2 dz = 1,
   * which gives alpha = 3 sqrt(2/beta) = 6 sqrt(2) at beta = 1/4. */
  o->eps = P->width * sqrt(P->beta / 2.0);
  o->alpha = 3.0 * sqrt(2.0 / P->beta);
  o->kcap = o->alpha / o->eps;
  /* M = dt Gamma (tau_g - 1/2), Sec. II below Eq. 16 */
  o->Gam = P->mobility / (P->tau_g - 0.5);
}

OAPI int orc_sizeof_params(void) { return (int)sizeof(orc_params); }

/* Number of OpenMP threads the per-site passes use (1 without OpenMP). */
OAPI int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Set the number of OpenMP threads of later passes (n >= 1); results do not
 * depend on it.  Returns the number in effect. */
OAPI int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

OAPI orc *orc_create(const orc_params *P, const double *Twall_bot,
                     const double *Twall_top) {
  if (P->wx < 1 || P->wy < 1 || P->NX < 1 || P->NY < 1) return NULL;
  orc *o = (orc *)calloc(1, sizeof(orc));
  o->P = *P;
  derive(o);
  o->n = P->wx * P->wy;
  const size_t n = (size_t)o->n;
  o->F = (double *)calloc(27 * n, sizeof(double));
  o->Fp = (double *)calloc(27 * n, sizeof(double));
  o->nb_kind = (int *)calloc(9 * n, sizeof(int));
  o->nb_loc = (int *)calloc(9 * n, sizeof(int));
  o->nb_col = (int *)calloc(9 * n, sizeof(int));
  for (int j = 0; j < P->wy; ++j)
    for (int i = 0; i < P->wx; ++i)
      for (int k = 1; k < NQ; ++k) {
        const size_t q = (size_t)k * n + (size_t)j * P->wx + i;
        int loc, gcol;
        o->nb_kind[q] = neighbour(o, i, j, OX[k], OY[k], &loc, &gcol);
        o->nb_loc[q] = loc;
        o->nb_col[q] = gcol;
      }
  o->Twb = (double *)calloc((size_t)P->NX, sizeof(double));
  o->Twt = (double *)calloc((size_t)P->NX, sizeof(double));
  double **fields[] = {&o->c,   &o->T,   &o->p,   &o->jx,  &o->jy,  &o->gcx,
                       &o->gcy, &o->lapc, &o->gTx, &o->gTy, &o->gpx, &o->gpy,
                       &o->mu,  &o->Fx,  &o->Fy,  &o->ux,  &o->uy,  &o->hxx,
                       &o->hxy, &o->hyy};
  for (size_t k = 0; k < sizeof(fields) / sizeof(fields[0]); ++k)
    *fields[k] = (double *)calloc(n, sizeof(double));
  if (Twall_bot) memcpy(o->Twb, Twall_bot, sizeof(double) * (size_t)P->NX);
  if (Twall_top) memcpy(o->Twt, Twall_top, sizeof(double) * (size_t)P->NX);
  return o;
}

OAPI void orc_destroy(orc *o) {
  if (!o) return;
  double *fields[] = {o->F,   o->Fp,  o->Twb, o->Twt, o->c,   o->T,
                      o->p,   o->jx,  o->jy,  o->gcx, o->gcy, o->lapc,
                      o->gTx, o->gTy, o->gpx, o->gpy, o->mu,  o->Fx,
                      o->Fy,  o->ux,  o->uy,  o->hxx, o->hxy, o->hyy};
  for (size_t k = 0; k < sizeof(fields) / sizeof(fields[0]); ++k) free(fields[k]);
  free(o->nb_kind);
  free(o->nb_loc);
  free(o->nb_col);
  free(o);
}

/* Initial state (the paper does not state one; READING): u = 0, p = p0,
 * c0 = (1 + phi0)/2, mu0 from c0 and its Laplacian, and every distribution
 * at its equilibrium for these fields: f = w p0 (Eq. 7), g from Eqs. 13-14,
 * hbar = w rho cv T0 (Eq. 22). */
OAPI void orc_init(orc *o, const double *phi0, const double *T0) {
  const orc_params *P = &o->P;
  const int n = o->n;
  for (int s = 0; s < n; ++s) o->c[s] = 0.5 * (1.0 + phi0[s]);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < P->wy; ++j)
    for (int i = 0; i < P->wx; ++i) {
      const int s = j * P->wx + i;
      double st[10];
      stencil_site(o, o->c, NULL, NULL, i, j, st);
      const double c = o->c[s];
      const double mu = mu_bulk(P->beta, c) - o->eps * o->eps * st[2];
      for (int k = 0; k < NQ; ++k) {
        o->F[k * n + s] = OW[k] * P->p0;
        const double H = (k == 0) ? (c - (1.0 - OW[0]) * o->Gam * mu / OCS2) / OW[0]
                                  : o->Gam * mu / OCS2;
        o->F[(NQ + k) * n + s] = OW[k] * H;
        o->F[(2 * NQ + k) * n + s] = OW[k] * rho_of(P, c) * P->cv * T0[s];
      }
    }
}

OAPI void orc_set_state(orc *o, const double *F) {
  memcpy(o->F, F, sizeof(double) * 27 * (size_t)o->n);
}

OAPI void orc_get_state(const orc *o, double *F) {
  memcpy(F, o->F, sizeof(double) * 27 * (size_t)o->n);
}

/* Diagnostics of the current state (needs passes A-C done). */
static void diag_from_passes(const orc *o, double *d) {
  const orc_params *P = &o->P;
  for (int k = 0; k < ORC_D_N; ++k) d[k] = 0.0;
  for (int j = 0; j < P->wy; ++j)
    for (int i = 0; i < P->wx; ++i) {
      const int s = j * P->wx + i;
      const double c = o->c[s];
      const double y = (double)(P->y0 + j) + 0.5;
      const double x = (double)(P->x0 + i) + 0.5;
      d[ORC_D_MASS] += c;
      d[ORC_D_ENERGY] += rho_of(P, c) * P->cv * o->T[s];
      d[ORC_D_SUM_CY] += c * y;
      d[ORC_D_SUM_CX] += c * x;
      /* u_r of Sec. IV C: sums over the sites with c >= 1/2 */
      if (c >= 0.5) {
        d[ORC_D_MASS_THR] += c;
        d[ORC_D_CUY_THR] += c * o->uy[s];
      }
      const double chk = c + o->T[s] + o->p[s] + o->ux[s] + o->uy[s];
      if (!isfinite(chk)) d[ORC_D_NONFINITE] += 1.0;
    }
}

/* Advance the state by nsteps: F_{n+1} = Stream(Collide(F_n)). */
OAPI void orc_step(orc *o, int nsteps) {
  for (int t = 0; t < nsteps; ++t) {
    pass_moments(o);
    pass_stencils(o);
    pass_closures(o);
    pass_pressure(o);
    pass_collide(o);
    pass_stream(o);
  }
}

/* Macroscopic fields of the current state: phi = 2c - 1, u, p, T.  Any
 * output pointer may be NULL. */
OAPI void orc_fields(orc *o, double *phi, double *ux, double *uy, double *p,
                     double *T) {
  pass_moments(o);
  pass_stencils(o);
  pass_closures(o);
  pass_pressure(o);
  for (int s = 0; s < o->n; ++s) {
    if (phi) phi[s] = 2.0 * o->c[s] - 1.0;
    if (ux) ux[s] = o->ux[s];
    if (uy) uy[s] = o->uy[s];
    if (p) p[s] = o->p[s];
    if (T) T[s] = o->T[s];
  }
}

/* Every intermediate field of the current state, 20 arrays of n in the order
 * c T p jx jy gcx gcy lapc gTx gTy gpx gpy mu Fx Fy ux uy hxx hxy hyy. */
OAPI void orc_intermediates(orc *o, double *out) {
  pass_moments(o);
  pass_stencils(o);
  pass_closures(o);
  pass_pressure(o);
  const double *src[] = {o->c,   o->T,   o->p,    o->jx,  o->jy,  o->gcx,
                         o->gcy, o->lapc, o->gTx, o->gTy, o->gpx, o->gpy,
                         o->mu,  o->Fx,  o->Fy,   o->ux,  o->uy,
                         o->hxx, o->hxy, o->hyy};
  for (int k = 0; k < 20; ++k)
    memcpy(out + (size_t)k * o->n, src[k], sizeof(double) * (size_t)o->n);
}

OAPI void orc_diag(orc *o, double *d) {
  pass_moments(o);
  pass_stencils(o);
  pass_closures(o);
  pass_pressure(o);
  diag_from_passes(o, d);
}

/* Single-site collision for pinning: in[27] pre-collision values at the site,
 * st[10] = (gcx, gcy, lapc, gTx, gTy, gpx, gpy, hxx, hxy, hyy) stencil values
 * (the Hessian of c is read by the curvature form only); writes out[27]
 * and aux[11] = (c, T, p, mu, Fx, Fy, ux, uy, wf, wT, wg), p being the
 * pressure of Eq. 9. */
OAPI void orc_collide_site(const orc_params *P, const double *in,
                           const double *st, double *out, double *aux) {
  orc o;
  memset(&o, 0, sizeof(o));
  o.P = *P;
  derive(&o);
  double c = 0, T = 0, p = 0, jx = 0, jy = 0;
  for (int k = 0; k < NQ; ++k) {
    p += in[k];
    jx += OX[k] * in[k];
    jy += OY[k] * in[k];
    c += in[NQ + k];
    T += in[2 * NQ + k];
  }
  T /= rho_of(P, c) * P->cv;
  closure_t r;
  closure_site(&o, c, T, jx, jy, st[0], st[1], st[2], st[3], st[4], st[5], st[6],
               st[7], st[8], st[9], &r);
  p += 0.5 * OCS2 * (r.ux * r.grx + r.uy * r.gry);   /* Eq. 9 */
  collide_site(&o, in, c, T, p, &r, out);
  if (aux) {
    aux[0] = c; aux[1] = T; aux[2] = p; aux[3] = r.mu; aux[4] = r.Fx;
    aux[5] = r.Fy; aux[6] = r.ux; aux[7] = r.uy; aux[8] = r.wf; aux[9] = r.wT;
    aux[10] = r.wg;
  }
}

/* Derived constants (eps, alpha, kcap, Gamma) for inspection by tests. */
OAPI void orc_derived(const orc_params *P, double *out4) {
  orc o;
  memset(&o, 0, sizeof(o));
  o.P = *P;
  derive(&o);
  out4[0] = o.eps; out4[1] = o.alpha; out4[2] = o.kcap; out4[3] = o.Gam;
}
