/* Oracle, two-dimensional reduced model (f, g) -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain serial-order FP64 implementation of the cut-cell method of
 * Dechriste & Mieussens (2015), written from the paper:
 *   velocity grid and discrete moments ......... Section 3.1, eq. (MacroscopicDDv)
 *   reduced BGK equilibria ..................... Section 2.2, eq. (BGKDD)
 *   reduced Shakhov equilibria ................. Section 2.2, eq. (ShakhovDD)
 *   level set, cell types, lengths, normal ..... Appendix A.1-A.2
 *   master search (fusion) and eq. (ii) ........ Appendix A.3
 *   virtual-cell and control-volume areas ...... Appendix A.4
 *   merge / scheme / redistribution ............ Section 3.3, eqs. (FusionDD),
 *                                                (ExSchemeDD), (FluxDD), (UpdateDD)
 *   discrete diffuse wall ...................... Section 3.3.1, eq. (BoundaryDDv)
 *   force, torque, wall stress, wall velocity .. Section 3.3.3, eqs. (eq-force),
 *                                                (eq-torque), (StressTensorDD), (uwDD)
 *   rigid-body update .......................... eqs. (motionDD_posit), (motionDD_vit)
 *   seven-step summary ......................... Section 3.3.4
 *   relaxation time from Kn .................... Section 5.3 (BGK, tau(Kn))
 *
 * Readings taken where the paper is silent or garbled are marked READING.
 * Nothing here is blocked, fused or reordered for speed: loops run over
 * cells, then members, then velocities.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define GAS 0
#define CUT 1
#define SOLID 2

typedef struct {
  int *type, *master;               /* master = -1 for solid cells */
  double *lxm, *lxp, *lym, *lyp;     /* gas lengths of the four Cartesian edges */
  double *lw, *nwx, *nwy, *rwx, *rwy;/* wall edge: length, normal into solid, centre */
  double *sbar, *scv;                /* virtual-cell area, control-volume area */
  int *mptr, *midx;                  /* members of each master, CSR, ascending */
} geo2d;

struct orc2d {
  orc_cfg cfg;
  int nx, ny, ncell, N, nvel;
  double dx, dy, dv, w, dt;
  double *v;                         /* N velocity nodes per axis */
  double *phi;                       /* vertex level set, (nx+1)*(ny+1) */
  geo2d g[2];                        /* geometry at t^n and t^{n+1} */
  int cur;
  /* rigid body state at t^n */
  double c[2], th, u[2], om;
};

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */
static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }

/* Reduced Maxwellian M[rho,u,T](v) = rho/(2 pi R T) exp(-|v-u|^2/(2 R T)),
   R = 1 (Section 2.2). */
static double maxw2(double rho, double ux, double uy, double T, double vx,
                    double vy) {
  double cx = vx - ux, cy = vy - uy;
  return rho / (2.0 * M_PI * T) * exp(-(cx * cx + cy * cy) / (2.0 * T));
}

/* Relaxation time of the BGK model from the Knudsen number:
   tau = sqrt(pi)/2 * (rho0/rho) * Kn L / sqrt(2 R T0), rho0 = R = T0 = 1. */
static double tau_of(const orc2d *o, double rho) {
  return sqrt(M_PI) / 2.0 * (1.0 / rho) * o->cfg.kn * o->cfg.lref / sqrt(2.0);
}

/* ------------------------------------------------------------------ */
/* level set (Appendix A): analytic signed distance, gas side positive */
/* ------------------------------------------------------------------ */

/* Distance from (x, y) to the ellipse x^2/a^2 + y^2/b^2 = 1, signed
   (negative inside).  The nearest point is (a^2 x/(t+a^2), b^2 y/(t+b^2))
   where t is the root of F(t) = (a x/(t+a^2))^2 + (b y/(t+b^2))^2 - 1,
   decreasing on t > -min(a,b)^2; the root is bracketed and bisected to the
   last bit (READING: "signed distance" of an ellipse taken as the exact
   Euclidean distance). */
static double ellipse_sdist(double a, double b, double x, double y) {
  double X = fabs(x), Y = fabs(y);
  if (a < b) { double t = a; a = b; b = t; t = X; X = Y; Y = t; }
  /* now a >= b, first quadrant */
  double inside = (X * X) / (a * a) + (Y * Y) / (b * b) - 1.0;
  double sgn = inside < 0.0 ? -1.0 : 1.0;
  double px, py;
  if (Y > 0.0) {
    if (X > 0.0) {
      double lo = -b * b, hi = sqrt(a * a * X * X + b * b * Y * Y) - b * b;
      if (hi < lo) hi = lo;
      /* make sure F(hi) <= 0 */
      for (int it = 0; it < 200; ++it) {
        double ra = a * X / (hi + a * a), rb = b * Y / (hi + b * b);
        if (ra * ra + rb * rb - 1.0 <= 0.0) break;
        hi = hi + fabs(hi) + 1.0;
      }
      for (int it = 0; it < 400; ++it) {
        double t = 0.5 * (lo + hi);
        if (t == lo || t == hi) break;
        double ra = a * X / (t + a * a), rb = b * Y / (t + b * b);
        double F = ra * ra + rb * rb - 1.0;
        if (F > 0.0) lo = t; else if (F < 0.0) hi = t; else { lo = hi = t; break; }
      }
      double t = 0.5 * (lo + hi);
      px = a * a * X / (t + a * a);
      py = b * b * Y / (t + b * b);
    } else {
      px = 0.0; py = b;
    }
  } else {
    /* on the major axis */
    double num = a * X, den = a * a - b * b;
    if (num < den) {
      double xa = num / den;
      px = a * xa; py = b * sqrt(dmax(0.0, 1.0 - xa * xa));
    } else {
      px = a; py = 0.0;
    }
  }
  double d = sqrt((px - X) * (px - X) + (py - Y) * (py - Y));
  return sgn * d;
}

static double levelset(const orc_cfg *cf, double cx, double cy, double th,
                       double x, double y) {
  double dxp = x - cx, dyp = y - cy;
  switch (cf->body_kind) {
    case 1: return sqrt(dxp * dxp + dyp * dyp) - cf->axes[0];
    case 2: {
      double ct = cos(th), st = sin(th);
      double xb = ct * dxp + st * dyp, yb = -st * dxp + ct * dyp; /* R(-theta)(x-c) */
      return ellipse_sdist(cf->axes[0], cf->axes[1], xb, yb);
    }
    case 3: return cf->axes[0] - sqrt(dxp * dxp + dyp * dyp);
    case 4: return dxp * cos(th) + dyp * sin(th);
    default: return 1.0e300;
  }
}

/* ------------------------------------------------------------------ */
/* geometry (Appendix A)                                               */
/* ------------------------------------------------------------------ */
static void geo_alloc(geo2d *g, int n) {
  g->type = calloc(n, sizeof(int));
  g->master = calloc(n, sizeof(int));
  g->mptr = calloc(n + 1, sizeof(int));
  g->midx = calloc(n, sizeof(int));
  double **d[] = {&g->lxm, &g->lxp, &g->lym, &g->lyp, &g->lw, &g->nwx,
                  &g->nwy, &g->rwx, &g->rwy, &g->sbar, &g->scv};
  for (unsigned k = 0; k < sizeof(d) / sizeof(d[0]); ++k) *d[k] = calloc(n, sizeof(double));
}

static void geo_free(geo2d *g) {
  free(g->type); free(g->master); free(g->mptr); free(g->midx);
  free(g->lxm); free(g->lxp); free(g->lym); free(g->lyp); free(g->lw);
  free(g->nwx); free(g->nwy); free(g->rwx); free(g->rwy); free(g->sbar);
  free(g->scv);
}

/* Gas length of one Cartesian edge from s = 0 (level set pa) to s = h
   (level set pb), and the crossing abscissa when exactly one end is gas.
   Crossing by linear interpolation: s = -h pa/(pb - pa) (Appendix A.2).
   READING: the printed length formula adds the full edge when both ends are
   gas on top of the two partial terms; the partial terms are used only when
   the ends differ (mixed edge), the full edge only when both are gas. */
static double edge_length(double pa, double pb, double h, int *mixed, double *sc) {
  int Ia = pa > 0.0, Ib = pb > 0.0;
  *mixed = (Ia != Ib);
  if (Ia && Ib) return h;
  if (!Ia && !Ib) return 0.0;
  double s = -h * pa / (pb - pa);
  *sc = s;
  return Ia ? fabs(s - 0.0) : fabs(h - s);
}

static int build_geometry(orc2d *o, geo2d *g, double cx, double cy, double th) {
  const orc_cfg *cf = &o->cfg;
  int nx = o->nx, ny = o->ny;
  double dx = o->dx, dy = o->dy;
  double eps = 1e-10 * dx;
  /* vertex level set with the clamp phi := sign(phi) max(|phi|, 1e-10 dx);
     READING: sign(0) := +1, a vertex on the boundary counts as gas. */
  for (int b = 0; b <= ny; ++b)
    for (int a = 0; a <= nx; ++a) {
      double x = cf->lo[0] + a * dx, y = cf->lo[1] + b * dy;
      double p = levelset(cf, cx, cy, th, x, y);
      double s = p >= 0.0 ? 1.0 : -1.0;
      o->phi[b * (nx + 1) + a] = s * dmax(fabs(p), eps);
    }
#define PHI(a, b) o->phi[(b) * (nx + 1) + (a)]
  int bad = 0;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int c = j * nx + i;
      double pmm = PHI(i, j), ppm = PHI(i + 1, j), ppp = PHI(i + 1, j + 1),
             pmp = PHI(i, j + 1);
      double m = dmin(dmin(pmm, ppm), dmin(ppp, pmp));
      double M = dmax(dmax(pmm, ppm), dmax(ppp, pmp));
      int type = m > 0.0 ? GAS : (M < 0.0 ? SOLID : CUT);
      g->type[c] = type;
      /* local coordinates relative to the lower-left vertex x_{i-1/2,j-1/2} */
      int mxp = 0, mxm = 0, myp = 0, mym = 0;
      double sxp = 0, sxm = 0, syp = 0, sym = 0;
      double Lxp = edge_length(ppm, ppp, dy, &mxp, &sxp);  /* right edge, along y */
      double Lxm = edge_length(pmm, pmp, dy, &mxm, &sxm);  /* left edge, along y */
      double Lyp = edge_length(pmp, ppp, dx, &myp, &syp);  /* top edge, along x */
      double Lym = edge_length(pmm, ppm, dx, &mym, &sym);  /* bottom edge, along x */
      g->lxp[c] = Lxp; g->lxm[c] = Lxm; g->lyp[c] = Lyp; g->lym[c] = Lym;
      int nmixed = mxp + mxm + myp + mym;
      if (nmixed == 4) bad = 1;  /* READING: two boundary pieces in one cell -> reject */
      /* crossing points (local coordinates) on mixed edges */
      double cxs[4], cys[4];
      int nc = 0;
      if (mxp) { cxs[nc] = dx; cys[nc] = sxp; ++nc; }
      if (mxm) { cxs[nc] = 0.0; cys[nc] = sxm; ++nc; }
      if (myp) { cxs[nc] = syp; cys[nc] = dy; ++nc; }
      if (mym) { cxs[nc] = sym; cys[nc] = 0.0; ++nc; }
      /* wall edge by closure of the virtual cell (Green formula for the
         normal).  READING: the printed Green normal points into the gas; the
         flux and the wall condition need the normal pointing into the wall,
         so n_w = -(dLx, dLy)/|L_w| with |L_w| = |(dLx, dLy)|, which is the
         chord length between the two crossings in exact arithmetic. */
      double dLx = Lxp - Lxm, dLy = Lyp - Lym;
      double Lw = sqrt(dLx * dLx + dLy * dLy);
      double nx_ = 0.0, ny_ = 0.0, rx = 0.0, ry = 0.0;
      if (type == CUT && nc == 2 && Lw > 0.0) {
        nx_ = -dLx / Lw; ny_ = -dLy / Lw;
        rx = 0.5 * (cxs[0] + cxs[1]); ry = 0.5 * (cys[0] + cys[1]);
      } else {
        Lw = 0.0;
      }
      g->lw[c] = Lw; g->nwx[c] = nx_; g->nwy[c] = ny_;
      g->rwx[c] = cf->lo[0] + i * dx + rx;
      g->rwy[c] = cf->lo[1] + j * dy + ry;
      /* area by the Green formula (Appendix A.4): sum over edges of
         1/4 |L| (sum of the edge's two end points) . outward normal.
         Left and bottom edges lie on x = 0 and y = 0 locally. */
      int Ipm = ppm > 0, Ipp = ppp > 0, Imp = pmp > 0;
      double S = 0.0;
      S += 0.25 * Lxp * ((Ipp ? dx : 0.0) + (Ipm ? dx : 0.0) + (mxp ? dx : 0.0));
      S += 0.25 * Lyp * ((Ipp ? dy : 0.0) + (Imp ? dy : 0.0) + (myp ? dy : 0.0));
      if (Lw > 0.0) S += 0.25 * Lw * ((cxs[0] + cxs[1]) * nx_ + (cys[0] + cys[1]) * ny_);
      g->sbar[c] = type == SOLID ? 0.0 : S;
    }
  /* master search, algorithm (fusion) with test (ii).  READING: the four
     tests are exclusive, in the order x+, x-, y+, y-, lengths within 1e-12
     of the maximum count as equal; more than 4 hops or a revisited cell
     rejects the geometry. */
  double thr = 1e-12 * dx;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int c = j * nx + i;
      if (g->type[c] == SOLID) { g->master[c] = -1; continue; }
      int ii = i, jj = j, hops = 0, visited[5];
      visited[0] = c;
      for (;;) {
        int cc = jj * nx + ii;
        double avg = 0.25 * (PHI(ii, jj) + PHI(ii + 1, jj) + PHI(ii + 1, jj + 1) + PHI(ii, jj + 1));
        if (avg > thr) break;
        /* READING: only edges shared with a cell of the domain can be chosen */
        double Lxp = ii + 1 < nx ? g->lxp[cc] : 0.0, Lxm = ii > 0 ? g->lxm[cc] : 0.0;
        double Lyp = jj + 1 < ny ? g->lyp[cc] : 0.0, Lym = jj > 0 ? g->lym[cc] : 0.0;
        double Mx = dmax(dmax(Lxp, Lxm), dmax(Lyp, Lym));
        double tie = Mx * (1.0 - 1e-12);
        if (Mx <= 0.0) { bad = 1; break; }
        if (Lxp >= tie) ii += 1;
        else if (Lxm >= tie) ii -= 1;
        else if (Lyp >= tie) jj += 1;
        else jj -= 1;
        if (ii < 0 || jj < 0 || ii >= nx || jj >= ny) { bad = 1; break; }
        ++hops;
        int nc = jj * nx + ii;
        for (int h = 0; h < hops; ++h) if (visited[h] == nc) bad = 1;
        if (hops > 4 || bad) { bad = 1; break; }
        visited[hops] = nc;
      }
      g->master[c] = jj * nx + ii;
    }
#undef PHI
  if (bad) return -3;
  /* members of each control volume, ascending cell index, and its area */
  int n = o->ncell;
  memset(g->mptr, 0, (n + 1) * sizeof(int));
  for (int c = 0; c < n; ++c) if (g->master[c] >= 0) g->mptr[g->master[c] + 1]++;
  for (int c = 0; c < n; ++c) g->mptr[c + 1] += g->mptr[c];
  int *fill = calloc(n, sizeof(int));
  for (int c = 0; c < n; ++c) {
    int m = g->master[c];
    if (m >= 0) g->midx[g->mptr[m] + fill[m]++] = c;
  }
  free(fill);
  for (int c = 0; c < n; ++c) {
    g->scv[c] = 0.0;
    for (int k = g->mptr[c]; k < g->mptr[c + 1]; ++k) g->scv[c] += g->sbar[g->midx[k]];
  }
  /* a master must be a cell whose centre is in the gas: it owns itself */
  for (int c = 0; c < n; ++c) {
    int m = g->master[c];
    if (m >= 0 && g->master[m] != m) return -3;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* creation                                                            */
/* ------------------------------------------------------------------ */
int orc2d_create(const orc_cfg *cfg, orc2d **out) {
  if (!cfg || cfg->dim != 2 || cfg->n[0] < 1 || cfg->n[1] < 1 || cfg->nv < 1 ||
      !(cfg->vmax > cfg->vmin))
    return -1;
  orc2d *o = calloc(1, sizeof(orc2d));
  if (!o) return -2;
  o->cfg = *cfg;
  o->nx = cfg->n[0]; o->ny = cfg->n[1]; o->ncell = o->nx * o->ny;
  o->N = cfg->nv; o->nvel = o->N * o->N;
  o->dx = (cfg->hi[0] - cfg->lo[0]) / o->nx;
  o->dy = (cfg->hi[1] - cfg->lo[1]) / o->ny;
  /* velocity grid (Section 3.1).  READING: nodes at cell midpoints of the
     velocity box, v_p = vmin + (p + 1/2) dv, so the grid is symmetric. */
  o->dv = (cfg->vmax - cfg->vmin) / o->N;
  o->w = o->dv * o->dv;
  o->v = malloc(o->N * sizeof(double));
  for (int p = 0; p < o->N; ++p) o->v[p] = cfg->vmin + (p + 0.5) * o->dv;
  /* time step.  READING: dt = CFL / (max|v_x|/dx + max|v_y|/dy), the simple
     form of the positivity condition (eq-CFL) with the constant folded into
     the CFL number. */
  double vm = 0.0;
  for (int p = 0; p < o->N; ++p) vm = dmax(vm, fabs(o->v[p]));
  o->dt = cfg->dt > 0.0 ? cfg->dt : cfg->cfl / (vm / o->dx + vm / o->dy);
  o->phi = malloc((size_t)(o->nx + 1) * (o->ny + 1) * sizeof(double));
  geo_alloc(&o->g[0], o->ncell);
  geo_alloc(&o->g[1], o->ncell);
  o->cur = 0;
  o->c[0] = cfg->center[0]; o->c[1] = cfg->center[1]; o->th = cfg->theta;
  o->u[0] = cfg->vel[0]; o->u[1] = cfg->vel[1]; o->om = cfg->omega;
  int st = build_geometry(o, &o->g[0], o->c[0], o->c[1], o->th);
  if (st) { orc2d_destroy(o); return st; }
  *out = o;
  return 0;
}

void orc2d_destroy(orc2d *o) {
  if (!o) return;
  free(o->v); free(o->phi);
  geo_free(&o->g[0]); geo_free(&o->g[1]);
  free(o);
}

double orc2d_dt(const orc2d *o) { return o->dt; }

void orc2d_velocity(const orc2d *o, double *v) { memcpy(v, o->v, o->N * sizeof(double)); }

void orc2d_geometry(const orc2d *o, int *type, int *master, double *lxm,
                    double *lxp, double *lym, double *lyp, double *lw,
                    double *nwx, double *nwy, double *rwx, double *rwy,
                    double *sbar, double *scv) {
  const geo2d *g = &o->g[o->cur];
  size_t n = o->ncell;
  memcpy(type, g->type, n * sizeof(int));
  memcpy(master, g->master, n * sizeof(int));
  memcpy(lxm, g->lxm, n * 8); memcpy(lxp, g->lxp, n * 8);
  memcpy(lym, g->lym, n * 8); memcpy(lyp, g->lyp, n * 8);
  memcpy(lw, g->lw, n * 8); memcpy(nwx, g->nwx, n * 8); memcpy(nwy, g->nwy, n * 8);
  memcpy(rwx, g->rwx, n * 8); memcpy(rwy, g->rwy, n * 8);
  memcpy(sbar, g->sbar, n * 8); memcpy(scv, g->scv, n * 8);
}

void orc2d_body_state(const orc2d *o, double *s) {
  s[0] = o->c[0]; s[1] = o->c[1]; s[2] = o->th; s[3] = o->u[0]; s[4] = o->u[1];
  s[5] = o->om;
}

/* READING: the initial state is the inflow Maxwellian in every non-solid
   cell, g = (R T/2) f; solid cells hold zero. */
void orc2d_init(const orc2d *o, double *f, double *g) {
  const double *in = o->cfg.inflow;
  const geo2d *G = &o->g[o->cur];
  for (int c = 0; c < o->ncell; ++c)
    for (int p2 = 0; p2 < o->N; ++p2)
      for (int p1 = 0; p1 < o->N; ++p1) {
        int p = p2 * o->N + p1;
        double M = maxw2(in[0], in[1], in[2], in[4], o->v[p1], o->v[p2]);
        size_t k = (size_t)c * o->nvel + p;
        f[k] = G->type[c] == SOLID ? 0.0 : M;
        g[k] = G->type[c] == SOLID ? 0.0 : 0.5 * in[4] * M;
      }
}

/* ------------------------------------------------------------------ */
/* merge over control volumes, eq. (FusionDD):                          */
/*   f_CV = (1/S_CV) sum_{k in sigma} Sbar_k f_k, written to all members */
/* ------------------------------------------------------------------ */
static void merge_with(const orc2d *o, const geo2d *G, double *f, double *g) {
  int nvel = o->nvel;
  double *accf = malloc(nvel * sizeof(double)), *accg = malloc(nvel * sizeof(double));
  for (int m = 0; m < o->ncell; ++m) {
    if (G->master[m] != m) continue;
    int b = G->mptr[m], e = G->mptr[m + 1];
    if (e - b <= 1) continue;  /* a control volume of one virtual cell: f_CV = f */
    for (int p = 0; p < nvel; ++p) { accf[p] = 0.0; accg[p] = 0.0; }
    for (int k = b; k < e; ++k) {
      int c = G->midx[k];
      for (int p = 0; p < nvel; ++p) {
        accf[p] += G->sbar[c] * f[(size_t)c * nvel + p];
        accg[p] += G->sbar[c] * g[(size_t)c * nvel + p];
      }
    }
    for (int k = b; k < e; ++k) {
      int c = G->midx[k];
      for (int p = 0; p < nvel; ++p) {
        f[(size_t)c * nvel + p] = accf[p] / G->scv[m];
        g[(size_t)c * nvel + p] = accg[p] / G->scv[m];
      }
    }
  }
  free(accf); free(accg);
}

void orc2d_merge(const orc2d *o, double *f, double *g) { merge_with(o, &o->g[o->cur], f, g); }

/* discrete moments of one cell, eq. (MacroscopicDDv): rho, rho u, E */
static void cell_moments(const orc2d *o, const double *f, const double *g,
                         double *rho, double *ux, double *uy, double *T) {
  double r = 0, mx = 0, my = 0, E = 0;
  for (int p2 = 0; p2 < o->N; ++p2)
    for (int p1 = 0; p1 < o->N; ++p1) {
      int p = p2 * o->N + p1;
      double vx = o->v[p1], vy = o->v[p2];
      r += f[p] * o->w;
      mx += vx * f[p] * o->w;
      my += vy * f[p] * o->w;
      E += 0.5 * (vx * vx + vy * vy) * f[p] * o->w + g[p] * o->w;
    }
  *rho = r; *ux = mx / r; *uy = my / r;
  /* E = rho|u|^2/2 + 3/2 rho R T (Section 2.1), R = 1 */
  *T = (2.0 * E / r - (*ux * *ux + *uy * *uy)) / 3.0;
}

/* Small dense solve A x = b (Gaussian elimination, partial pivoting); A and
   b are overwritten, x returned in b.  n <= 5. */
static int solve_small(int n, double A[5][5], double *b) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int r = k + 1; r < n; ++r)
      if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
    if (A[piv][k] == 0.0) return -1;
    if (piv != k) {
      for (int c = 0; c < n; ++c) { double t = A[k][c]; A[k][c] = A[piv][c]; A[piv][c] = t; }
      double t = b[k]; b[k] = b[piv]; b[piv] = t;
    }
    for (int r = k + 1; r < n; ++r) {
      double m = A[r][k] / A[k][k];
      for (int c = k; c < n; ++c) A[r][c] -= m * A[k][c];
      b[r] -= m * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int c = k + 1; c < n; ++c) s -= A[k][c] * b[c];
    b[k] = s / A[k][k];
  }
  return 0;
}

/* Conservative equilibrium (Section 3.1, the Newton algorithm of Titarev):
   the triplet (rho, u, T) of the equilibrium pair (M, G = T/2 M) is the root
   of  sum_p psi_p (M_p, G_p) w = sum_p psi_p (f_p, g_p) w  for the
   collision invariants psi = (1, v_x, v_y, |v|^2/2 for M and 1 for G),
   so that the discrete relaxation term conserves mass, momentum and energy
   exactly.  Newton from the directly computed triplet; the Jacobian is the
   sum of psi times the derivatives of (M, G) in (rho, u_x, u_y, T).
   Once a step is below 1e-13 of (rho, sqrt T, T) one more step is taken
   (quadratic convergence puts the iterate at the rounding floor) and the
   iteration stops.  Returns the iterations taken, -1 without convergence in
   50 iterations. */
static int conservative_triplet2(const orc2d *o, const double *f, const double *g,
                                 double *x /* rho, ux, uy, T in/out */) {
  int N = o->N;
  double target[4] = {0, 0, 0, 0};
  for (int p = 0; p < o->nvel; ++p) {
    double vx = o->v[p % N], vy = o->v[p / N];
    target[0] += f[p] * o->w;
    target[1] += vx * f[p] * o->w;
    target[2] += vy * f[p] * o->w;
    target[3] += (0.5 * (vx * vx + vy * vy) * f[p] + g[p]) * o->w;
  }
  int polish = 0;
  for (int it = 1; it <= 50; ++it) {
    double r = x[0], ux = x[1], uy = x[2], T = x[3];
    double R[5] = {0, 0, 0, 0, 0}, J[5][5];
    memset(J, 0, sizeof(J));
    for (int p = 0; p < o->nvel; ++p) {
      double vx = o->v[p % N], vy = o->v[p / N];
      double cx = vx - ux, cy = vy - uy;
      double M = maxw2(r, ux, uy, T, vx, vy);
      double dM[4] = {M / r, M * cx / T, M * cy / T, M * ((cx * cx + cy * cy) / (2.0 * T * T) - 1.0 / T)};
      double psi[4] = {1.0, vx, vy, 0.5 * (vx * vx + vy * vy)};
      for (int i = 0; i < 4; ++i) {
        R[i] += psi[i] * M * o->w;
        for (int j = 0; j < 4; ++j) J[i][j] += psi[i] * dM[j] * o->w;
      }
      /* energy carried by G = T/2 M */
      R[3] += 0.5 * T * M * o->w;
      for (int j = 0; j < 4; ++j) J[3][j] += 0.5 * T * dM[j] * o->w;
      J[3][3] += 0.5 * M * o->w;
    }
    for (int i = 0; i < 4; ++i) R[i] -= target[i];
    if (solve_small(4, J, R)) return -1;
    for (int i = 0; i < 4; ++i) x[i] -= R[i];
    if (polish) return it;
    double su = sqrt(fabs(x[3]));
    if (fabs(R[0]) <= 1e-13 * fabs(x[0]) && fabs(R[1]) <= 1e-13 * su &&
        fabs(R[2]) <= 1e-13 * su && fabs(R[3]) <= 1e-13 * fabs(x[3]))
      polish = 1;
  }
  return -1;
}

/* triplet of the relaxation of one cell: direct moments, or conservative */
static int equilibrium2(const orc2d *o, const double *f, const double *g, double *rho,
                        double *ux, double *uy, double *T) {
  cell_moments(o, f, g, rho, ux, uy, T);
  if (!o->cfg.maxwellian) return 0;
  double x[4] = {*rho, *ux, *uy, *T};
  int it = conservative_triplet2(o, f, g, x);
  /* READING: a cell whose iteration does not converge keeps the direct triplet */
  if (it > 0) { *rho = x[0]; *ux = x[1]; *uy = x[2]; *T = x[3]; }
  return it;
}

int orc2d_equilibrium(const orc2d *o, const double *f, const double *g, double *out) {
  int it = equilibrium2(o, f, g, &out[0], &out[1], &out[2], &out[3]);
  return it;
}

/* What the relaxation of one cell relaxes toward: the triplet above and, for
   the Shakhov model, the heat flux q of eq. (MacroscopicDDv).  READING: q is
   taken about the directly computed mean velocity, as printed, also when the
   conservative equilibrium supplies the triplet. */
typedef struct { double rho, ux, uy, T, qx, qy; } relax2;

static void relax_target2(const orc2d *o, const double *f, const double *g, relax2 *t) {
  equilibrium2(o, f, g, &t->rho, &t->ux, &t->uy, &t->T);
  t->qx = t->qy = 0.0;
  if (o->cfg.model != 1) return;
  double r, ux, uy, T;
  cell_moments(o, f, g, &r, &ux, &uy, &T);
  double qx = 0.0, qy = 0.0;
  for (int p2 = 0; p2 < o->N; ++p2)
    for (int p1 = 0; p1 < o->N; ++p1) {
      int p = p2 * o->N + p1;
      double cx = o->v[p1] - ux, cy = o->v[p2] - uy;
      double h = 0.5 * (cx * cx + cy * cy) * f[p] + g[p];
      qx += cx * h * o->w;
      qy += cy * h * o->w;
    }
  t->qx = qx; t->qy = qy;
}

/* Reduced equilibria at (vx, vy): eq. (BGKDD), or eq. (ShakhovDD) with the
   pressure P = rho R T, R = 1. */
static void equilibrium_at2(const orc2d *o, const relax2 *t, double vx, double vy, double *fe,
                            double *ge) {
  double M = maxw2(t->rho, t->ux, t->uy, t->T, vx, vy);
  if (o->cfg.model != 1) { *fe = M; *ge = 0.5 * t->T * M; return; }
  double cx = vx - t->ux, cy = vy - t->uy, c2 = cx * cx + cy * cy;
  double P = t->rho * t->T;
  double s = (1.0 - o->cfg.prandtl) * (cx * t->qx + cy * t->qy) / (5.0 * P * t->T);
  *fe = M * (1.0 + s * (c2 / t->T - 4.0));
  *ge = 0.5 * t->T * M * (1.0 + s * (c2 / t->T - 2.0));
}

void orc2d_equilibrium_values(const orc2d *o, const double *f, const double *g, double *fe,
                              double *ge) {
  relax2 t;
  relax_target2(o, f, g, &t);
  for (int p = 0; p < o->nvel; ++p)
    equilibrium_at2(o, &t, o->v[p % o->N], o->v[p / o->N], &fe[p], &ge[p]);
}

/* wall velocity of the boundary point r, eq. (uwDD) */
static void wall_velocity(const orc2d *o, double rx, double ry, double *uwx, double *uwy) {
  double ax = rx - o->c[0], ay = ry - o->c[1];
  *uwx = o->u[0] + (-ay) * o->om;
  *uwy = o->u[1] + (ax) * o->om;
}

/* wall density and wall distribution of one wall edge, eq. (BoundaryDDv):
   phi_w = - sum_{c>0} c f_CV dv / sum_{c<0} c M[1,u_w,T_w] dv,
   f_w = phi_w M_w, g_w = phi_w (R T_w / 2) M_w.  READING: the g factor is
   R T_w / 2 (the wall temperature). */
static void wall_state(const orc2d *o, const double *fcv, double nx_, double ny_,
                       double uwx, double uwy, double *fw, double *gw) {
  double Tw = o->cfg.t_wall, num = 0.0, den = 0.0;
  for (int p2 = 0; p2 < o->N; ++p2)
    for (int p1 = 0; p1 < o->N; ++p1) {
      int p = p2 * o->N + p1;
      double cn = (o->v[p1] - uwx) * nx_ + (o->v[p2] - uwy) * ny_;
      if (cn > 0.0) num += cn * fcv[p] * o->w;
      else if (cn < 0.0) den += cn * maxw2(1.0, uwx, uwy, Tw, o->v[p1], o->v[p2]) * o->w;
    }
  double phiw = den != 0.0 ? -num / den : 0.0;
  for (int p2 = 0; p2 < o->N; ++p2)
    for (int p1 = 0; p1 < o->N; ++p1) {
      int p = p2 * o->N + p1;
      double Mw = maxw2(1.0, uwx, uwy, Tw, o->v[p1], o->v[p2]);
      fw[p] = phiw * Mw;
      gw[p] = phiw * 0.5 * Tw * Mw;
    }
}

/* farfield ghost value (READING: outer faces see the inflow Maxwellian) */
static double ghost_f(const orc2d *o, int p) {
  const double *in = o->cfg.inflow;
  return maxw2(in[0], in[1], in[2], in[4], o->v[p % o->N], o->v[p / o->N]);
}

/* Scheme (ExSchemeDD) for the control volume of master m with the fluxes
   (FluxDD) of its members at t^n (geometry G) and the area ratio
   S^n / S^{n+1,*}; result written to fo/go (nvel each). */
static void scheme_cv(const orc2d *o, const geo2d *G, const double *fm,
                      const double *gm, int m, double snew, double *fo, double *go,
                      double *fw, double *gw) {
  int nvel = o->nvel, N = o->N, nx = o->nx, ny = o->ny;
  double dt = o->dt;
  const double *fc = fm + (size_t)m * nvel, *gc = gm + (size_t)m * nvel;
  double S = G->scv[m];
  /* READING: with the conservative equilibrium the whole triplet, rho in
     the relaxation time included, comes from the Newton solution */
  relax2 tg;
  relax_target2(o, fc, gc, &tg);
  double rho = tg.rho;
  int collide = o->cfg.kn > 0.0;
  double tau = collide ? tau_of(o, rho) : 1.0;
  /* transport residual R_p = sum over members of (F_x+ - F_x-) + (F_y+ - F_y-) + F_w */
  double *R = calloc(nvel, sizeof(double)), *Rg = calloc(nvel, sizeof(double));
  for (int kk = G->mptr[m]; kk < G->mptr[m + 1]; ++kk) {
    int k = G->midx[kk];
    int i = k % nx, j = k / nx;
    int has_wall = G->lw[k] > 0.0;
    double uwx = 0, uwy = 0;
    if (has_wall) {
      wall_velocity(o, G->rwx[k], G->rwy[k], &uwx, &uwy);
      wall_state(o, fc, G->nwx[k], G->nwy[k], uwx, uwy, fw, gw);
    }
    const double *fk = fm + (size_t)k * nvel, *gk = gm + (size_t)k * nvel;
    for (int p = 0; p < nvel; ++p) {
      double vx = o->v[p % N], vy = o->v[p / N];
      /* neighbour values: the neighbour cell's value, or the farfield ghost */
      double fe, ge, fwst, gwst, fn, gn, fs, gs;
      if (i + 1 < nx) { fe = fm[(size_t)(k + 1) * nvel + p]; ge = gm[(size_t)(k + 1) * nvel + p]; }
      else { fe = ghost_f(o, p); ge = 0.5 * o->cfg.inflow[4] * fe; }
      if (i > 0) { fwst = fm[(size_t)(k - 1) * nvel + p]; gwst = gm[(size_t)(k - 1) * nvel + p]; }
      else { fwst = ghost_f(o, p); gwst = 0.5 * o->cfg.inflow[4] * fwst; }
      if (j + 1 < ny) { fn = fm[(size_t)(k + nx) * nvel + p]; gn = gm[(size_t)(k + nx) * nvel + p]; }
      else { fn = ghost_f(o, p); gn = 0.5 * o->cfg.inflow[4] * fn; }
      if (j > 0) { fs = fm[(size_t)(k - nx) * nvel + p]; gs = gm[(size_t)(k - nx) * nvel + p]; }
      else { fs = ghost_f(o, p); gs = 0.5 * o->cfg.inflow[4] * fs; }
      double vxm = dmin(vx, 0.0), vxp = dmax(vx, 0.0);
      double vym = dmin(vy, 0.0), vyp = dmax(vy, 0.0);
      double Fxp = G->lxp[k] * (vxm * fe + vxp * fk[p]);
      double Fxm = G->lxm[k] * (vxm * fk[p] + vxp * fwst);
      double Fyp = G->lyp[k] * (vym * fn + vyp * fk[p]);
      double Fym = G->lym[k] * (vym * fk[p] + vyp * fs);
      double Gxp = G->lxp[k] * (vxm * ge + vxp * gk[p]);
      double Gxm = G->lxm[k] * (vxm * gk[p] + vxp * gwst);
      double Gyp = G->lyp[k] * (vym * gn + vyp * gk[p]);
      double Gym = G->lym[k] * (vym * gk[p] + vyp * gs);
      double Fw = 0.0, Gw = 0.0;
      if (has_wall) {
        double cn = (vx - uwx) * G->nwx[k] + (vy - uwy) * G->nwy[k];
        Fw = G->lw[k] * (dmin(cn, 0.0) * fw[p] + dmax(cn, 0.0) * fk[p]);
        Gw = G->lw[k] * (dmin(cn, 0.0) * gw[p] + dmax(cn, 0.0) * gk[p]);
      }
      R[p] += (Fxp - Fxm) + (Fyp - Fym) + Fw;
      Rg[p] += (Gxp - Gxm) + (Gyp - Gym) + Gw;
    }
  }
  if (o->cfg.scheme == 1) {
    /* Semi-implicit scheme (ImpSchemeDD): explicit transport, then the
       relaxation toward the equilibrium of t^{n+1} taken implicitly.  Its
       moments follow from summing the scheme over the velocities, where the
       collision term vanishes: they are those of the transported value.
       READING: tau^n comes from the directly computed density of the
       control volume at t^n. */
    double *fs = calloc(nvel, sizeof(double)), *gs = calloc(nvel, sizeof(double));
    double ratio = S / snew;
    for (int p = 0; p < nvel; ++p) {
      fs[p] = ratio * fc[p] - dt / snew * R[p];
      gs[p] = ratio * gc[p] - dt / snew * Rg[p];
    }
    double rn, uxn, uyn, Tn;
    cell_moments(o, fc, gc, &rn, &uxn, &uyn, &Tn);
    double nu = collide ? dt / tau_of(o, rn) : 0.0;
    relax2 t1;
    relax_target2(o, fs, gs, &t1);
    for (int p = 0; p < nvel; ++p) {
      double E = 0.0, Ge = 0.0;
      if (collide) equilibrium_at2(o, &t1, o->v[p % N], o->v[p / N], &E, &Ge);
      fo[p] = (fs[p] + nu * E) / (1.0 + nu);
      go[p] = (gs[p] + nu * Ge) / (1.0 + nu);
    }
    free(fs); free(gs); free(R); free(Rg);
    return;
  }
  for (int p = 0; p < nvel; ++p) {
    double vx = o->v[p % N], vy = o->v[p / N];
    double E = 0.0, Ge = 0.0;
    if (collide) equilibrium_at2(o, &tg, vx, vy, &E, &Ge);   /* eq. (BGKDD) / (ShakhovDD) */
    double ratio = S / snew;
    double fnew = ratio * fc[p] - dt / snew * R[p];
    double gnew = ratio * gc[p] - dt / snew * Rg[p];
    if (collide) {
      fnew += ratio * (dt / tau) * (E - fc[p]);
      gnew += ratio * (dt / tau) * (Ge - gc[p]);
    }
    fo[p] = fnew; go[p] = gnew;
  }
  free(R); free(Rg);
}

void orc2d_update_cells(const orc2d *o, const double *fm, const double *gm,
                        const int *cells, int ncells, double *fo, double *go) {
  const geo2d *G = &o->g[o->cur];
  int nvel = o->nvel;
#pragma omp parallel
  {
    double *fw = malloc(nvel * sizeof(double)), *gw = malloc(nvel * sizeof(double));
#pragma omp for schedule(dynamic, 4)
    for (int q = 0; q < ncells; ++q) {
      int c = cells[q];
      double *fq = fo + (size_t)q * nvel, *gq = go + (size_t)q * nvel;
      int m = G->master[c];
      if (m < 0) {
        for (int p = 0; p < nvel; ++p) { fq[p] = 0.0; gq[p] = 0.0; }
        continue;
      }
      scheme_cv(o, G, fm, gm, m, G->scv[m], fq, gq, fw, gw);
    }
    free(fw); free(gw);
  }
}

/* Wall stress (StressTensorDD) times the normal, summed into force and
   torque (eq-force), (eq-torque), plus the mass of the state (def-masse).
   READING: drag = x-component of the force on the body; torque about the
   body centre, a x b = a_x b_y - a_y b_x. */
static void force_with(const orc2d *o, const geo2d *G, const double *fm,
                       const double *gm, double *diag) {
  int nvel = o->nvel, N = o->N;
  double *fw = malloc(nvel * sizeof(double)), *gw = malloc(nvel * sizeof(double));
  double Fx = 0.0, Fy = 0.0, Tq = 0.0, mass = 0.0;
  for (int k = 0; k < o->ncell; ++k) {
    if (G->lw[k] <= 0.0) continue;
    int m = G->master[k];
    const double *fc = fm + (size_t)m * nvel;
    double uwx, uwy;
    wall_velocity(o, G->rwx[k], G->rwy[k], &uwx, &uwy);
    wall_state(o, fc, G->nwx[k], G->nwy[k], uwx, uwy, fw, gw);
    double sx = 0.0, sy = 0.0;  /* Sigma_w n_w */
    for (int p = 0; p < nvel; ++p) {
      double cx = o->v[p % N] - uwx, cy = o->v[p / N] - uwy;
      double cn = cx * G->nwx[k] + cy * G->nwy[k];
      double fv = cn < 0.0 ? fw[p] : (cn > 0.0 ? fc[p] : 0.0);
      sx += cx * cn * fv * o->w;
      sy += cy * cn * fv * o->w;
    }
    Fx += sx * G->lw[k];
    Fy += sy * G->lw[k];
    double ax = G->rwx[k] - o->c[0], ay = G->rwy[k] - o->c[1];
    Tq += (ax * sy - ay * sx) * G->lw[k];
  }
  for (int m = 0; m < o->ncell; ++m) {
    if (G->master[m] != m) continue;
    double s = 0.0;
    for (int p = 0; p < nvel; ++p) s += fm[(size_t)m * nvel + p] * o->w;
    mass += G->scv[m] * s;
  }
  (void)gm;
  diag[0] = Fx; diag[1] = Fy; diag[2] = Tq; diag[3] = mass;
  free(fw); free(gw);
}

void orc2d_force(const orc2d *o, const double *fm, const double *gm, double *diag) {
  force_with(o, &o->g[o->cur], fm, gm, diag);
}

/* ------------------------------------------------------------------ */
/* one time step (Section 3.3.4, seven steps)                          */
/* ------------------------------------------------------------------ */
int orc2d_step(orc2d *o, const double *f, const double *g, double *fo,
               double *go, double *diag) {
  int n = o->ncell, nvel = o->nvel;
  size_t tot = (size_t)n * nvel;
  geo2d *Gn = &o->g[o->cur];
  int moving = o->cfg.motion != 0 && o->cfg.body_kind != 0;
  double *fm = malloc(tot * sizeof(double)), *gm = malloc(tot * sizeof(double));
  memcpy(fm, f, tot * sizeof(double));
  memcpy(gm, g, tot * sizeof(double));

  /* 1. body position at t^{n+1}, eq. (motionDD_posit) */
  double c1[2] = {o->c[0] + o->dt * o->u[0], o->c[1] + o->dt * o->u[1]};
  double th1 = o->th + o->dt * o->om;
  /* 2. merge over the control volumes of t^n, eq. (FusionDD) */
  merge_with(o, Gn, fm, gm);
  /* 3. geometry at t^{n+1} and areas S^{n+1,*} over sigma^n */
  geo2d *G1 = Gn;
  double *snew = malloc(n * sizeof(double));
  int *target = malloc(n * sizeof(int));   /* control volume of t^n receiving each cell */
  for (int c = 0; c < n; ++c) { snew[c] = Gn->scv[c]; target[c] = Gn->master[c]; }
  if (moving) {
    G1 = &o->g[1 - o->cur];
    int st = build_geometry(o, G1, c1[0], c1[1], th1);
    if (st) { free(fm); free(gm); free(snew); free(target); return st; }
    /* READING: a cell solid at t^n and gas or cut at t^{n+1} (appearing)
       joins the control volume of t^n reached by hopping across its largest
       edge at t^{n+1}; it adds 0 to S^n and its new area to S^{n+1,*}. */
    int nx = o->nx;
    for (int c = 0; c < n; ++c) {
      if (!(Gn->type[c] == SOLID && G1->type[c] != SOLID)) continue;
      int cc = c, hops = 0;
      while (Gn->master[cc] < 0 && hops < 4) {
        int i = cc % nx, j = cc / nx;
        double Lxp = i + 1 < nx ? G1->lxp[cc] : 0.0, Lxm = i > 0 ? G1->lxm[cc] : 0.0;
        double Lyp = j + 1 < o->ny ? G1->lyp[cc] : 0.0, Lym = j > 0 ? G1->lym[cc] : 0.0;
        double Mx = dmax(dmax(Lxp, Lxm), dmax(Lyp, Lym)), tie = Mx * (1.0 - 1e-12);
        if (Lxp >= tie) i += 1; else if (Lxm >= tie) i -= 1;
        else if (Lyp >= tie) j += 1; else j -= 1;
        if (i < 0 || j < 0 || i >= nx || j >= o->ny) break;
        cc = j * nx + i;
        ++hops;
      }
      if (Gn->master[cc] < 0) { free(fm); free(gm); free(snew); free(target); return -3; }
      target[c] = Gn->master[cc];
    }
    for (int c = 0; c < n; ++c) snew[c] = 0.0;
    for (int c = 0; c < n; ++c)
      if (target[c] >= 0) snew[target[c]] += G1->sbar[c];
  }
  /* 4-5. wall condition at t^n, force and torque from the wall stress, then
     the body velocities at t^{n+1}, eq. (motionDD_vit) */
  double dg[4];
  force_with(o, Gn, fm, gm, dg);
  if (diag) memcpy(diag, dg, sizeof(dg));
  /* 6-7. scheme on every control volume of t^n, then redistribution to the
     virtual cells of t^{n+1} merged into it, eq. (UpdateDD) */
  double *fcv = malloc(tot * sizeof(double)), *gcv = malloc(tot * sizeof(double));
#pragma omp parallel
  {
    double *fw = malloc(nvel * sizeof(double)), *gw = malloc(nvel * sizeof(double));
#pragma omp for schedule(dynamic, 16)
    for (int m = 0; m < n; ++m) {
      if (Gn->master[m] != m || snew[m] <= 0.0) continue;
      scheme_cv(o, Gn, fm, gm, m, snew[m], fcv + (size_t)m * nvel,
                gcv + (size_t)m * nvel, fw, gw);
    }
    free(fw); free(gw);
  }
  for (int c = 0; c < n; ++c) {
    int m = target[c];
    double *fd = fo + (size_t)c * nvel, *gd = go + (size_t)c * nvel;
    if (m < 0 || snew[m] <= 0.0 || G1->type[c] == SOLID) {
      memset(fd, 0, nvel * sizeof(double));
      memset(gd, 0, nvel * sizeof(double));
    } else {
      memcpy(fd, fcv + (size_t)m * nvel, nvel * sizeof(double));
      memcpy(gd, gcv + (size_t)m * nvel, nvel * sizeof(double));
    }
  }
  free(fcv); free(gcv);
  if (moving) {
    /* rigid body: explicit Euler for position (with the old velocity) and
       velocity (with the force of t^n).  READING (free rotation): the centre
       is pinned, only the rotation responds to the torque. */
    if (o->cfg.motion == 1) {
      o->om = o->om + o->dt * dg[2] / o->cfg.inertia;
    }
    o->c[0] = c1[0]; o->c[1] = c1[1]; o->th = th1;
    o->cur = 1 - o->cur;
  }
  free(fm); free(gm); free(snew); free(target);
  return 0;
}

/* moments of every cell, eq. (MacroscopicDDv): rho, u, T, Sigma, q */
void orc2d_moments(const orc2d *o, const double *f, const double *g, double *out) {
  int nvel = o->nvel, N = o->N;
  for (int c = 0; c < o->ncell; ++c) {
    const double *fc = f + (size_t)c * nvel, *gc = g + (size_t)c * nvel;
    double *q = out + (size_t)c * 9;
    if (o->g[o->cur].type[c] == SOLID) { for (int k = 0; k < 9; ++k) q[k] = 0.0; continue; }
    double rho, ux, uy, T;
    cell_moments(o, fc, gc, &rho, &ux, &uy, &T);
    double sxx = 0, sxy = 0, syy = 0, qx = 0, qy = 0;
    for (int p = 0; p < nvel; ++p) {
      double cx = o->v[p % N] - ux, cy = o->v[p / N] - uy;
      sxx += cx * cx * fc[p] * o->w;
      sxy += cx * cy * fc[p] * o->w;
      syy += cy * cy * fc[p] * o->w;
      double h = 0.5 * (cx * cx + cy * cy) * fc[p] + gc[p];
      qx += cx * h * o->w;
      qy += cy * h * o->w;
    }
    q[0] = rho; q[1] = ux; q[2] = uy; q[3] = T;
    q[4] = sxx; q[5] = sxy; q[6] = syy; q[7] = qx; q[8] = qy;
  }
}

#ifdef _OPENMP
#include <omp.h>
#endif
/* number of threads the oracle's parallel loops use */
int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* threads for the parallel loops from now on (the single-thread baseline) */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Adjoint of the fixed-geometry step (not in the paper: the transpose  */
/* of the scheme above, written out term by term).                     */
/*                                                                     */
/* With x^n the merged state entering step n and Lambda^{n+1}_m the    */
/* sensitivity of the objective to the value that control volume m     */
/* writes to its members, the adjoint step accumulates                 */
/*   a^n = sum_m (d Phi_m / d x^n)^T Lambda^{n+1}_m                     */
/* per cell, and Lambda^n_m = sum over the members j of m of a^n[j]    */
/* (the merge and the redistribution transpose into that sum).          */
/* Terms: identity and relaxation (1 - beta) with beta = dt rho / kappa;*/
/* the Jacobian of the Maxwellian through (rho, rho u, E); the upwind   */
/* fluxes transposed (outflow on the own value, inflow gathered onto    */
/* the upwind cell); the wall flux with its density phi_w linear in the */
/* outgoing part of x (rank one per wall edge).  Parameter partials     */
/* accumulate into dJ/dT_w, dJ/dKn and dJ/du (farfield faces and the    */
/* initial state).                                                      */
/* ------------------------------------------------------------------ */

/* weights of the objective per wall edge: drag (1, 0), torque (-a_y, a_x) */
static void obj_weights(const orc2d *o, const geo2d *G, int k, int objective,
                        double *al, double *ga) {
  if (objective == 0) { *al = 1.0; *ga = 0.0; return; }
  double ax = G->rwx[k] - o->c[0], ay = G->rwy[k] - o->c[1];
  *al = -ay; *ga = ax;
}

/* dJ/dx of the objective at a merged state, per cell (f only), plus dJ/dT_w */
static void objective_adjoint(const orc2d *o, const geo2d *G, const double *fm, int objective,
                              double *af, double *dTw) {
  int nvel = o->nvel, N = o->N;
  double Tw = o->cfg.t_wall, w = o->w;
  for (int k = 0; k < o->ncell; ++k) {
    if (G->lw[k] <= 0.0) continue;
    int m = G->master[k];
    const double *fc = fm + (size_t)m * nvel;
    double al, ga;
    obj_weights(o, G, k, objective, &al, &ga);
    double num = 0.0, den = 0.0, dden = 0.0;
    for (int p = 0; p < nvel; ++p) {
      double vx = o->v[p % N], vy = o->v[p / N];
      double cn = vx * G->nwx[k] + vy * G->nwy[k];
      double Mw = maxw2(1.0, 0.0, 0.0, Tw, vx, vy);
      if (cn > 0.0) num += cn * fc[p] * w;
      else if (cn < 0.0) {
        den += cn * Mw * w;
        dden += cn * Mw * ((vx * vx + vy * vy) / (2.0 * Tw * Tw) - 1.0 / Tw) * w;
      }
    }
    double phi = den != 0.0 ? -num / den : 0.0;
    double dphi = den != 0.0 ? num / (den * den) * dden : 0.0;
    /* sum over incoming velocities of psi c M_w w, and its T_w derivative */
    double sin_ = 0.0, sdT = 0.0;
    for (int p = 0; p < nvel; ++p) {
      double vx = o->v[p % N], vy = o->v[p / N];
      double cn = vx * G->nwx[k] + vy * G->nwy[k];
      if (cn >= 0.0) continue;
      double psi = al * vx + ga * vy;
      double Mw = maxw2(1.0, 0.0, 0.0, Tw, vx, vy);
      double dMw = Mw * ((vx * vx + vy * vy) / (2.0 * Tw * Tw) - 1.0 / Tw);
      sin_ += psi * cn * Mw * w;
      sdT += psi * cn * (dphi * Mw + phi * dMw) * w;
    }
    *dTw += G->lw[k] * sdT;
    for (int q = 0; q < nvel; ++q) {
      double vx = o->v[q % N], vy = o->v[q / N];
      double cn = vx * G->nwx[k] + vy * G->nwy[k];
      if (cn <= 0.0) continue;
      double psi = al * vx + ga * vy;
      af[(size_t)m * nvel + q] += G->lw[k] * (psi * cn * w + sin_ * (-cn * w / den));
    }
  }
}

/* one adjoint step: Lf, Lg = Lambda^{n+1} stored at master indices;
   af, ag (zeroed by the caller) receive a^n per cell; gp += partials
   (0: T_w, 1: Kn, 2: u_x, 3: u_y of the farfield) */
static void adjoint_step(const orc2d *o, const geo2d *G, const double *fm, const double *gm,
                         const double *Lf, const double *Lg, double *af, double *ag,
                         double *gp) {
  int nvel = o->nvel, N = o->N, nx = o->nx, ny = o->ny;
  double dt = o->dt, w = o->w, Tw = o->cfg.t_wall;
  const double *in = o->cfg.inflow;
  int collide = o->cfg.kn > 0.0;
  double kappa = sqrt(M_PI) / 2.0 * o->cfg.kn * o->cfg.lref / sqrt(2.0);
  for (int m = 0; m < o->ncell; ++m) {
    if (G->master[m] != m) continue;
    const double *lf = Lf + (size_t)m * nvel, *lg = Lg + (size_t)m * nvel;
    const double *fc = fm + (size_t)m * nvel, *gc = gm + (size_t)m * nvel;
    double S = G->scv[m];
    double rho, ux, uy, T;
    cell_moments(o, fc, gc, &rho, &ux, &uy, &T);
    double beta = collide ? dt * rho / kappa : 0.0;
    /* (i) identity, relaxation and the Maxwellian's Jacobian */
    for (int q = 0; q < nvel; ++q) {
      af[(size_t)m * nvel + q] += (1.0 - beta) * lf[q];
      ag[(size_t)m * nvel + q] += (1.0 - beta) * lg[q];
    }
    if (collide) {
      double s_r = 0, s_ux = 0, s_uy = 0, s_T = 0, C = 0;
      for (int p = 0; p < nvel; ++p) {
        double vx = o->v[p % N], vy = o->v[p / N];
        double cx = vx - ux, cy = vy - uy, c2 = cx * cx + cy * cy;
        double E = maxw2(rho, ux, uy, T, vx, vy);
        double dEr = E / rho, dEux = E * cx / T, dEuy = E * cy / T;
        double dET = E * (c2 / (2.0 * T * T) - 1.0 / T);
        s_r += lf[p] * dEr + lg[p] * 0.5 * T * dEr;
        s_ux += lf[p] * dEux + lg[p] * 0.5 * T * dEux;
        s_uy += lf[p] * dEuy + lg[p] * 0.5 * T * dEuy;
        s_T += lf[p] * dET + lg[p] * (0.5 * E + 0.5 * T * dET);
        C += lf[p] * (E - fc[p]) + lg[p] * (0.5 * T * E - gc[p]);
      }
      /* (rho, u, T) -> (rho, rho u, E) */
      double u2 = ux * ux + uy * uy;
      double A_r = s_r + s_ux * (-ux / rho) + s_uy * (-uy / rho) + s_T * (u2 - 3.0 * T) / (3.0 * rho);
      double A_px = s_ux / rho + s_T * (-2.0 * ux / (3.0 * rho));
      double A_py = s_uy / rho + s_T * (-2.0 * uy / (3.0 * rho));
      double A_e = s_T * 2.0 / (3.0 * rho);
      for (int q = 0; q < nvel; ++q) {
        double vx = o->v[q % N], vy = o->v[q / N];
        af[(size_t)m * nvel + q] += beta * w * (A_r + A_px * vx + A_py * vy + A_e * 0.5 * (vx * vx + vy * vy))
                                    + dt * w / kappa * C;
        ag[(size_t)m * nvel + q] += beta * w * A_e;
      }
      gp[1] += C * (-beta / o->cfg.kn);
    }
    /* (ii) fluxes of every edge of every member; (iii) wall edges */
    for (int kk = G->mptr[m]; kk < G->mptr[m + 1]; ++kk) {
      int k = G->midx[kk];
      int i = k % nx, j = k / nx;
      struct { double L; int nb; int axis; double sgn; } e[4] = {
          {G->lxp[k], i + 1 < nx ? k + 1 : -1, 0, 1.0},
          {G->lxm[k], i > 0 ? k - 1 : -1, 0, -1.0},
          {G->lyp[k], j + 1 < ny ? k + nx : -1, 1, 1.0},
          {G->lym[k], j > 0 ? k - nx : -1, 1, -1.0}};
      for (int f = 0; f < 4; ++f) {
        if (e[f].L == 0.0) continue;
        for (int q = 0; q < nvel; ++q) {
          double vd = e[f].axis == 0 ? o->v[q % N] : o->v[q / N];
          double c = e[f].sgn * vd;
          double cp = dmax(c, 0.0), cm = dmin(c, 0.0);
          double co = -dt / S * e[f].L;
          af[(size_t)k * nvel + q] += co * cp * lf[q];
          ag[(size_t)k * nvel + q] += co * cp * lg[q];
          if (e[f].nb >= 0) {
            af[(size_t)e[f].nb * nvel + q] += co * cm * lf[q];
            ag[(size_t)e[f].nb * nvel + q] += co * cm * lg[q];
          } else if (cm != 0.0) {
            /* farfield ghost M[rho, u, T] and T/2 of it: d/du_d = M (v_d - u_d)/T */
            double vx = o->v[q % N], vy = o->v[q / N];
            double M = maxw2(in[0], in[1], in[2], in[4], vx, vy);
            double t = co * cm * (lf[q] + 0.5 * in[4] * lg[q]);
            gp[2] += t * M * (vx - in[1]) / in[4];
            gp[3] += t * M * (vy - in[2]) / in[4];
          }
        }
      }
      if (G->lw[k] > 0.0) {
        double Lw = G->lw[k], co = -dt / S * Lw;
        double num = 0.0, den = 0.0, dden = 0.0;
        for (int p = 0; p < nvel; ++p) {
          double vx = o->v[p % N], vy = o->v[p / N];
          double cn = vx * G->nwx[k] + vy * G->nwy[k];
          double Mw = maxw2(1.0, 0.0, 0.0, Tw, vx, vy);
          if (cn > 0.0) num += cn * fc[p] * w;
          else if (cn < 0.0) {
            den += cn * Mw * w;
            dden += cn * Mw * ((vx * vx + vy * vy) / (2.0 * Tw * Tw) - 1.0 / Tw) * w;
          }
        }
        double phi = den != 0.0 ? -num / den : 0.0;
        double dphi = den != 0.0 ? num / (den * den) * dden : 0.0;
        double Lam = 0.0, dT = 0.0;
        for (int p = 0; p < nvel; ++p) {
          double vx = o->v[p % N], vy = o->v[p / N];
          double cn = vx * G->nwx[k] + vy * G->nwy[k];
          if (cn >= 0.0) continue;
          double Mw = maxw2(1.0, 0.0, 0.0, Tw, vx, vy);
          double dMw = Mw * ((vx * vx + vy * vy) / (2.0 * Tw * Tw) - 1.0 / Tw);
          Lam += cn * Mw * (lf[p] + 0.5 * Tw * lg[p]);
          double dfw = dphi * Mw + phi * dMw;
          double dgw = dphi * 0.5 * Tw * Mw + phi * (0.5 * Mw + 0.5 * Tw * dMw);
          dT += cn * (lf[p] * dfw + lg[p] * dgw);
        }
        gp[0] += co * dT;
        for (int q = 0; q < nvel; ++q) {
          double vx = o->v[q % N], vy = o->v[q / N];
          double cn = vx * G->nwx[k] + vy * G->nwy[k];
          if (cn <= 0.0) continue;
          af[(size_t)k * nvel + q] += co * cn * lf[q];
          ag[(size_t)k * nvel + q] += co * cn * lg[q];
          af[(size_t)m * nvel + q] += co * Lam * (-cn * w / den);
        }
      }
    }
  }
}

/* Lambda_m = sum over the members j of m of a[j], stored at m */
static void cv_sum(const orc2d *o, const geo2d *G, const double *a, double *L) {
  int nvel = o->nvel;
  memset(L, 0, (size_t)o->ncell * nvel * sizeof(double));
  for (int c = 0; c < o->ncell; ++c) {
    int m = G->master[c];
    if (m < 0) continue;
    for (int p = 0; p < nvel; ++p) L[(size_t)m * nvel + p] += a[(size_t)c * nvel + p];
  }
}

/* Runs nsteps from the inflow Maxwellian, J = objective (0 drag, 1 torque)
   of the final state, and its gradient: out = J, dJ/dT_w, dJ/dKn, dJ/du_x,
   dJ/du_y (u = farfield velocity). Fixed bodies only. */
int orc2d_adjoint(orc2d *o, int nsteps, int objective, double *out) {
  if (o->cfg.motion != 0 && o->cfg.body_kind != 0) return -1;
  if (o->cfg.maxwellian || o->cfg.scheme || o->cfg.model) return -1;   /* transpose written for the explicit direct BGK step */
  if (nsteps < 1) return -1;
  int nvel = o->nvel, N = o->N;
  size_t tot = (size_t)o->ncell * nvel;
  const geo2d *G = &o->g[o->cur];
  double **F = malloc((nsteps + 1) * sizeof(double *)), **Gs = malloc((nsteps + 1) * sizeof(double *));
  for (int n = 0; n <= nsteps; ++n) { F[n] = malloc(tot * 8); Gs[n] = malloc(tot * 8); }
  orc2d_init(o, F[0], Gs[0]);
  for (int n = 0; n < nsteps; ++n) orc2d_step(o, F[n], Gs[n], F[n + 1], Gs[n + 1], NULL);
  /* merged states x^n */
  for (int n = 0; n <= nsteps; ++n) merge_with(o, G, F[n], Gs[n]);
  double diag[4];
  force_with(o, G, F[nsteps], Gs[nsteps], diag);
  double J = objective == 0 ? diag[0] : diag[2];
  double *af = calloc(tot, 8), *ag = calloc(tot, 8), *Lf = calloc(tot, 8), *Lg = calloc(tot, 8);
  double gp[4] = {0, 0, 0, 0};
  objective_adjoint(o, G, F[nsteps], objective, af, &gp[0]);
  for (int n = nsteps - 1; n >= 0; --n) {
    cv_sum(o, G, af, Lf);
    cv_sum(o, G, ag, Lg);
    memset(af, 0, tot * 8); memset(ag, 0, tot * 8);
    adjoint_step(o, G, F[n], Gs[n], Lf, Lg, af, ag, gp);
  }
  /* initial state: every non-solid cell holds M[rho, u, T] (and T/2 of it) */
  cv_sum(o, G, af, Lf);
  cv_sum(o, G, ag, Lg);
  const double *in = o->cfg.inflow;
  for (int m = 0; m < o->ncell; ++m) {
    if (G->master[m] != m) continue;
    for (int p = 0; p < nvel; ++p) {
      double vx = o->v[p % N], vy = o->v[p / N];
      double M = maxw2(in[0], in[1], in[2], in[4], vx, vy);
      double t = Lf[(size_t)m * nvel + p] + 0.5 * in[4] * Lg[(size_t)m * nvel + p];
      gp[2] += t * M * (vx - in[1]) / in[4];
      gp[3] += t * M * (vy - in[2]) / in[4];
    }
  }
  out[0] = J; out[1] = gp[0]; out[2] = gp[1]; out[3] = gp[2]; out[4] = gp[3];
  for (int n = 0; n <= nsteps; ++n) { free(F[n]); free(Gs[n]); }
  free(F); free(Gs); free(af); free(ag); free(Lf); free(Lg);
  return 0;
}
