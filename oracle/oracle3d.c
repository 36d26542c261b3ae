/* Oracle, three-dimensional model (F) -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain serial-order FP64 implementation of the 3D cut-cell method of
 * Dechriste & Mieussens (2015), Section 5 (fixed body):
 *   moments and Maxwellian ........................ Section 2.1, eqs. (MacroscopicTD), (MaxwellianTD)
 *   Shakhov equilibrium ........................... Section 2.1
 *   diffuse wall with zero net mass flux ........... Section 5 step 4
 *   explicit scheme with seven virtual faces ....... eq. (eq-schema3D)
 *   control volumes, merge, redistribution ......... Section 5 steps 2, 6, 7
 * READING (the paper leaves the 3D geometry "to the reader"): the gas area
 * of a Cartesian face is the 2D virtual-cell polygon of that face's four
 * vertices (linear crossings on mixed edges); the wall face closes the cell,
 * |S_w| n_w = -sum_k |S_k| n_k, n_w pointing into the solid; its centre is
 * the mean of the cell's edge crossings; the volume follows from the
 * divergence theorem, V = 1/3 sum_faces |S| (m . n).  READING (printed
 * typos of eq. eq-schema3D): the y and z fluxes use v_{p2} and v_{p3}, the
 * collision term carries dt, tau is per cell.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define GAS 0
#define CUT 1
#define SOLID 2

struct orc3d {
  orc_cfg cfg;
  int nx, ny, nz, ncell, N, nvel;
  double dx, dy, dz, dv, w, dt;
  double *v;
  double *phi;                    /* (nx+1)(ny+1)(nz+1) */
  int *type, *master, *mptr, *midx;
  double *S[6];                   /* gas areas of the faces x-, x+, y-, y+, z-, z+ */
  double *sw, *nw[3], *rw[3];     /* wall area, normal into the solid, centre */
  double *vbar, *vcv;             /* virtual-cell volume, control-volume volume */
};

static double mn(double a, double b) { return a < b ? a : b; }
static double mx(double a, double b) { return a > b ? a : b; }

/* 3D Maxwellian rho/(2 pi R T)^{3/2} exp(-|v-u|^2/(2 R T)), R = 1 */
static double maxw3(double rho, const double *u, double T, double vx, double vy, double vz) {
  double cx = vx - u[0], cy = vy - u[1], cz = vz - u[2];
  return rho / pow(2.0 * M_PI * T, 1.5) * exp(-(cx * cx + cy * cy + cz * cz) / (2.0 * T));
}

/* gas polygon of a rectangle [0,h1]x[0,h2] whose corners (0,0), (h1,0),
   (h1,h2), (0,h2) carry level-set values q[0..3]: area and centroid;
   *saddle set when all four edges are crossed */
static void face_polygon(const double *q, double h1, double h2, double *area, double *cs,
                         double *ct, int *saddle, int *ncross, double *xs, double *xt) {
  double cx[4] = {0, h1, h1, 0}, cy[4] = {0, 0, h2, h2};
  double ps[8], pt[8];
  int np = 0, nc = 0;
  for (int e = 0; e < 4; ++e) {
    int e1 = (e + 1) % 4;
    if (q[e] > 0.0) { ps[np] = cx[e]; pt[np] = cy[e]; ++np; }
    if ((q[e] > 0.0) != (q[e1] > 0.0)) {
      double t = q[e] / (q[e] - q[e1]);
      double s_ = cx[e] + t * (cx[e1] - cx[e]), t_ = cy[e] + t * (cy[e1] - cy[e]);
      ps[np] = s_; pt[np] = t_; ++np;
      xs[nc] = s_; xt[nc] = t_; ++nc;
    }
  }
  *saddle = nc == 4;
  *ncross = nc;
  double A = 0.0, Cs = 0.0, Ct = 0.0;
  for (int k = 0; k < np; ++k) {
    int k1 = (k + 1) % np;
    double cr = ps[k] * pt[k1] - ps[k1] * pt[k];
    A += cr;
    Cs += (ps[k] + ps[k1]) * cr;
    Ct += (pt[k] + pt[k1]) * cr;
  }
  A *= 0.5;
  *area = A;
  if (A > 0.0) { *cs = Cs / (6.0 * A); *ct = Ct / (6.0 * A); }
  else { *cs = 0.0; *ct = 0.0; }
}

/* Signed distance to the body, gas side positive (Appendix A), with the
   body turned by th about the z axis through its centre.
   5 sphere: radius axes[0].
   6 vane: the points within r = min(axes) of the box of half-sizes
     axes - r (body frame), i.e. a plate with rounded edges; the body frame
     is the frame turned by th.  Distance to the box: the length of the
     positive part of q = |p| - (axes - r) outside, the largest component of
     q inside; minus r. */
static double levelset3(const orc_cfg *cf, double th, double x, double y, double z) {
  double a = x - cf->center[0], b = y - cf->center[1], c = z - cf->center[2];
  if (cf->body_kind == 5) return sqrt(a * a + b * b + c * c) - cf->axes[0];
  if (cf->body_kind == 6) {
    double ct = cos(th), st = sin(th);
    double p[3] = {ct * a + st * b, -st * a + ct * b, c};
    double r = mn(cf->axes[0], mn(cf->axes[1], cf->axes[2]));
    double q[3], out2 = 0.0, qmax = -1e300;
    for (int d = 0; d < 3; ++d) {
      q[d] = fabs(p[d]) - (cf->axes[d] - r);
      out2 += mx(q[d], 0.0) * mx(q[d], 0.0);
      qmax = mx(qmax, q[d]);
    }
    return sqrt(out2) + mn(qmax, 0.0) - r;
  }
  return 1.0e300;
}

/* Geometry of one cell of sizes h[3] from its 8 clamped vertex values
   q8[a | b << 1 | c << 2] (a, b, c = 0/1 along x, y, z): type, the gas
   areas S6 of its faces (x-, x+, y-, y+, z-, z+), the wall area, its unit
   normal into the solid and its centre relative to the cell's lower corner,
   and the gas volume.  Returns 1 when a face is a saddle (four crossings). */
static int cell_geom3(const double *q8, const double *h, int *type_out, double *S6, double *sw_out,
                      double *nw_out, double *rloc, double *vbar) {
  double qmin = 1e300, qmax = -1e300;
  int bad = 0;
  for (int t = 0; t < 8; ++t) { qmin = mn(qmin, q8[t]); qmax = mx(qmax, q8[t]); }
  int type = qmin > 0.0 ? GAS : (qmax < 0.0 ? SOLID : CUT);
  *type_out = type;
  /* faces: axis d, side s (0: at 0, 1: at h_d); local axes (d1, d2) */
  double V = 0.0;
  double Aw[3] = {0, 0, 0};
  for (int d = 0; d < 3; ++d) {
    int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
    for (int sd = 0; sd < 2; ++sd) {
      double q[4];
      /* corners in the order (0,0), (h1,0), (h1,h2), (0,h2) of (d1, d2) */
      int co[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
      for (int t = 0; t < 4; ++t) {
        int idx[3];
        idx[d] = sd; idx[d1] = co[t][0]; idx[d2] = co[t][1];
        q[t] = q8[idx[0] | (idx[1] << 1) | (idx[2] << 2)];
      }
      double area, cs, ct, xs[4], xt[4];
      int saddle, ncr;
      face_polygon(q, h[d1], h[d2], &area, &cs, &ct, &saddle, &ncr, xs, xt);
      if (saddle) bad = 1;
      S6[2 * d + sd] = type == SOLID ? 0.0 : area;
      /* outward normal: -e_d on side 0, +e_d on side 1; m.n = sd*h_d */
      double sgn = sd ? 1.0 : -1.0;
      Aw[d] -= sgn * area;
      V += area * (sd ? h[d] : 0.0) / 3.0;
    }
  }
  /* edge crossings of the cell (12 edges) -> wall centre */
  double rs[3] = {0, 0, 0};
  int ncx = 0;
  for (int d = 0; d < 3; ++d)
    for (int t = 0; t < 4; ++t) {
      int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
      int idx0[3], idx1[3];
      idx0[d] = 0; idx1[d] = 1;
      idx0[d1] = idx1[d1] = t & 1;
      idx0[d2] = idx1[d2] = (t >> 1) & 1;
      double qa = q8[idx0[0] | (idx0[1] << 1) | (idx0[2] << 2)];
      double qb = q8[idx1[0] | (idx1[1] << 1) | (idx1[2] << 2)];
      if ((qa > 0.0) != (qb > 0.0)) {
        double tt = qa / (qa - qb);
        double p3[3];
        p3[d] = tt * h[d]; p3[d1] = idx0[d1] * h[d1]; p3[d2] = idx0[d2] * h[d2];
        rs[0] += p3[0]; rs[1] += p3[1]; rs[2] += p3[2];
        ++ncx;
      }
    }
  double Sw = sqrt(Aw[0] * Aw[0] + Aw[1] * Aw[1] + Aw[2] * Aw[2]);
  if (type == CUT && ncx > 0 && Sw > 0.0) {
    double r[3] = {rs[0] / ncx, rs[1] / ncx, rs[2] / ncx};
    *sw_out = Sw;
    for (int d = 0; d < 3; ++d) { nw_out[d] = Aw[d] / Sw; rloc[d] = r[d]; }
    V += (r[0] * Aw[0] + r[1] * Aw[1] + r[2] * Aw[2]) / 3.0;
  } else {
    *sw_out = 0.0;
    for (int d = 0; d < 3; ++d) { nw_out[d] = 0.0; rloc[d] = 0.0; }
  }
  *vbar = type == SOLID ? 0.0 : (type == GAS ? h[0] * h[1] * h[2] : V);
  return bad;
}

static int build3(orc3d *o) {
  const orc_cfg *cf = &o->cfg;
  int nx = o->nx, ny = o->ny, nz = o->nz;
  int vx = nx + 1, vy = ny + 1;
  double eps = 1e-10 * o->dx;
  for (int c = 0; c <= nz; ++c)
    for (int b = 0; b <= ny; ++b)
      for (int a = 0; a <= nx; ++a) {
        double p = levelset3(cf, cf->theta, cf->lo[0] + a * o->dx, cf->lo[1] + b * o->dy, cf->lo[2] + c * o->dz);
        double s = p >= 0.0 ? 1.0 : -1.0;
        o->phi[((size_t)c * vy + b) * vx + a] = s * mx(fabs(p), eps);
      }
#define PH(a, b, c) o->phi[((size_t)(c) * vy + (b)) * vx + (a)]
  int bad = 0;
  double h[3] = {o->dx, o->dy, o->dz};
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int cc = (k * ny + j) * nx + i;
        double q8[8];
        for (int t = 0; t < 8; ++t) q8[t] = PH(i + (t & 1), j + ((t >> 1) & 1), k + ((t >> 2) & 1));
        double S6[6], sw, nw[3], rl[3], vb;
        int type;
        if (cell_geom3(q8, h, &type, S6, &sw, nw, rl, &vb)) bad = 1;
        o->type[cc] = type;
        for (int f = 0; f < 6; ++f) o->S[f][cc] = S6[f];
        o->sw[cc] = sw;
        for (int d = 0; d < 3; ++d) o->nw[d][cc] = nw[d];
        if (sw > 0.0) {
          o->rw[0][cc] = cf->lo[0] + i * o->dx + rl[0];
          o->rw[1][cc] = cf->lo[1] + j * o->dy + rl[1];
          o->rw[2][cc] = cf->lo[2] + k * o->dz + rl[2];
        } else {
          for (int d = 0; d < 3; ++d) o->rw[d][cc] = 0.0;
        }
        o->vbar[cc] = vb;
      }
  /* masters: centre in gas = mean of the 8 vertex values > 1e-12 dx; hop
     across the largest face shared with a cell of the domain, order
     x+, x-, y+, y-, z+, z- */
  double thr = 1e-12 * o->dx;
  for (int cc = 0; cc < o->ncell; ++cc) {
    if (o->type[cc] == SOLID) { o->master[cc] = -1; continue; }
    int i = cc % nx, j = (cc / nx) % ny, k = cc / (nx * ny), hops = 0;
    int seen[5];
    seen[0] = cc;
    for (;;) {
      int c2 = (k * ny + j) * nx + i;
      double avg = 0.0;
      for (int t = 0; t < 8; ++t) avg += PH(i + (t & 1), j + ((t >> 1) & 1), k + ((t >> 2) & 1));
      if (avg / 8.0 > thr) break;
      double L[6] = {i + 1 < nx ? o->S[1][c2] : 0.0, i > 0 ? o->S[0][c2] : 0.0,
                     j + 1 < ny ? o->S[3][c2] : 0.0, j > 0 ? o->S[2][c2] : 0.0,
                     k + 1 < nz ? o->S[5][c2] : 0.0, k > 0 ? o->S[4][c2] : 0.0};
      double M = 0.0;
      for (int t = 0; t < 6; ++t) M = mx(M, L[t]);
      if (!(M > 0.0) || hops == 4) { bad = 1; break; }
      double tie = M * (1.0 - 1e-12);
      int t = 0;
      while (L[t] < tie) ++t;
      if (t == 0) i += 1; else if (t == 1) i -= 1; else if (t == 2) j += 1;
      else if (t == 3) j -= 1; else if (t == 4) k += 1; else k -= 1;
      ++hops;
      int nc = (k * ny + j) * nx + i;
      for (int hh = 0; hh < hops; ++hh) if (seen[hh] == nc) bad = 1;
      if (bad) break;
      seen[hops] = nc;
    }
    o->master[cc] = (k * ny + j) * nx + i;
  }
#undef PH
  if (bad) return -3;
  int n = o->ncell;
  memset(o->mptr, 0, (n + 1) * sizeof(int));
  for (int c = 0; c < n; ++c) if (o->master[c] >= 0) o->mptr[o->master[c] + 1]++;
  for (int c = 0; c < n; ++c) o->mptr[c + 1] += o->mptr[c];
  int *fill = calloc(n, sizeof(int));
  for (int c = 0; c < n; ++c) {
    int m = o->master[c];
    if (m >= 0) o->midx[o->mptr[m] + fill[m]++] = c;
  }
  free(fill);
  for (int c = 0; c < n; ++c) {
    o->vcv[c] = 0.0;
    for (int q = o->mptr[c]; q < o->mptr[c + 1]; ++q) o->vcv[c] += o->vbar[o->midx[q]];
  }
  for (int c = 0; c < n; ++c) {
    int m = o->master[c];
    if (m >= 0 && o->master[m] != m) return -3;
  }
  return 0;
}

void orc3d_destroy(orc3d *o);

int orc3d_create(const orc_cfg *cfg, orc3d **out) {
  if (!cfg || cfg->dim != 3 || cfg->n[0] < 1 || cfg->n[1] < 1 || cfg->n[2] < 1 || cfg->nv < 1 ||
      !(cfg->vmax > cfg->vmin))
    return -1;
  orc3d *o = calloc(1, sizeof(orc3d));
  o->cfg = *cfg;
  o->nx = cfg->n[0]; o->ny = cfg->n[1]; o->nz = cfg->n[2];
  o->ncell = o->nx * o->ny * o->nz;
  o->N = cfg->nv; o->nvel = o->N * o->N * o->N;
  o->dx = (cfg->hi[0] - cfg->lo[0]) / o->nx;
  o->dy = (cfg->hi[1] - cfg->lo[1]) / o->ny;
  o->dz = (cfg->hi[2] - cfg->lo[2]) / o->nz;
  o->dv = (cfg->vmax - cfg->vmin) / o->N;
  o->w = o->dv * o->dv * o->dv;
  o->v = malloc(o->N * sizeof(double));
  for (int p = 0; p < o->N; ++p) o->v[p] = cfg->vmin + (p + 0.5) * o->dv;
  double vm = 0.0;
  for (int p = 0; p < o->N; ++p) vm = mx(vm, fabs(o->v[p]));
  o->dt = cfg->dt > 0.0 ? cfg->dt : cfg->cfl / (vm / o->dx + vm / o->dy + vm / o->dz);
  size_t n = o->ncell;
  o->phi = malloc((size_t)(o->nx + 1) * (o->ny + 1) * (o->nz + 1) * sizeof(double));
  o->type = calloc(n, sizeof(int)); o->master = calloc(n, sizeof(int));
  o->mptr = calloc(n + 1, sizeof(int)); o->midx = calloc(n, sizeof(int));
  for (int f = 0; f < 6; ++f) o->S[f] = calloc(n, sizeof(double));
  o->sw = calloc(n, sizeof(double));
  for (int d = 0; d < 3; ++d) { o->nw[d] = calloc(n, sizeof(double)); o->rw[d] = calloc(n, sizeof(double)); }
  o->vbar = calloc(n, sizeof(double)); o->vcv = calloc(n, sizeof(double));
  int st = build3(o);
  if (st) { orc3d_destroy(o); return st; }
  *out = o;
  return 0;
}

void orc3d_destroy(orc3d *o) {
  if (!o) return;
  free(o->v); free(o->phi); free(o->type); free(o->master); free(o->mptr); free(o->midx);
  for (int f = 0; f < 6; ++f) free(o->S[f]);
  free(o->sw);
  for (int d = 0; d < 3; ++d) { free(o->nw[d]); free(o->rw[d]); }
  free(o->vbar); free(o->vcv);
  free(o);
}

double orc3d_dt(const orc3d *o) { return o->dt; }

/* geometry export: type, master, S (6 per cell, x-,x+,y-,y+,z-,z+), sw,
   nw (3 per cell), rw (3 per cell), vbar, vcv */
void orc3d_geometry(const orc3d *o, int *type, int *master, double *S6, double *sw, double *nw3,
                    double *rw3, double *vbar, double *vcv) {
  size_t n = o->ncell;
  memcpy(type, o->type, n * sizeof(int));
  memcpy(master, o->master, n * sizeof(int));
  for (size_t c = 0; c < n; ++c) {
    for (int f = 0; f < 6; ++f) S6[6 * c + f] = o->S[f][c];
    for (int d = 0; d < 3; ++d) { nw3[3 * c + d] = o->nw[d][c]; rw3[3 * c + d] = o->rw[d][c]; }
  }
  memcpy(sw, o->sw, n * 8); memcpy(vbar, o->vbar, n * 8); memcpy(vcv, o->vcv, n * 8);
}

void orc3d_init(const orc3d *o, double *F) {
  const double *in = o->cfg.inflow;
  double u[3] = {in[1], in[2], in[3]};
  int N = o->N;
  for (int c = 0; c < o->ncell; ++c)
    for (int p = 0; p < o->nvel; ++p) {
      double M = maxw3(in[0], u, in[4], o->v[p % N], o->v[(p / N) % N], o->v[p / (N * N)]);
      F[(size_t)c * o->nvel + p] = o->type[c] == SOLID ? 0.0 : M;
    }
}

static void merge3(const orc3d *o, double *F) {
  int nvel = o->nvel;
  double *acc = malloc(nvel * sizeof(double));
  for (int m = 0; m < o->ncell; ++m) {
    if (o->master[m] != m || o->mptr[m + 1] - o->mptr[m] <= 1) continue;
    for (int p = 0; p < nvel; ++p) acc[p] = 0.0;
    for (int q = o->mptr[m]; q < o->mptr[m + 1]; ++q) {
      int c = o->midx[q];
      for (int p = 0; p < nvel; ++p) acc[p] += o->vbar[c] * F[(size_t)c * nvel + p];
    }
    for (int q = o->mptr[m]; q < o->mptr[m + 1]; ++q) {
      int c = o->midx[q];
      for (int p = 0; p < nvel; ++p) F[(size_t)c * nvel + p] = acc[p] / o->vcv[m];
    }
  }
  free(acc);
}

void orc3d_merge(const orc3d *o, double *F) { merge3(o, F); }

static void moments3(const orc3d *o, const double *F, double *rho, double *u, double *T) {
  int N = o->N;
  double r = 0, m[3] = {0, 0, 0}, E = 0;
  for (int p = 0; p < o->nvel; ++p) {
    double vx = o->v[p % N], vy = o->v[(p / N) % N], vz = o->v[p / (N * N)];
    r += F[p] * o->w;
    m[0] += vx * F[p] * o->w; m[1] += vy * F[p] * o->w; m[2] += vz * F[p] * o->w;
    E += 0.5 * (vx * vx + vy * vy + vz * vz) * F[p] * o->w;
  }
  *rho = r;
  for (int d = 0; d < 3; ++d) u[d] = m[d] / r;
  /* E = rho |u|^2/2 + 3/2 rho R T */
  *T = (2.0 * E / r - (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])) / 3.0;
}

/* dense solve A x = b, n <= 5 (Gaussian elimination, partial pivoting) */
static int solve5(int n, double A[5][5], double *b) {
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

/* Conservative equilibrium (Section 3.1, Newton algorithm of Titarev) in
   3D: (rho, u, T) such that the discrete moments of the sampled Maxwellian
   for psi = (1, v, |v|^2/2) equal those of F.  Newton from the direct
   moments; once a step is below 1e-13 of (rho, sqrt T, T) one more step is
   taken and the iteration stops; -1 without convergence in 50 iterations. */
static int conservative_triplet3(const orc3d *o, const double *F, double *x /* rho u(3) T */) {
  int N = o->N;
  double target[5] = {0, 0, 0, 0, 0};
  for (int p = 0; p < o->nvel; ++p) {
    double v[3] = {o->v[p % N], o->v[(p / N) % N], o->v[p / (N * N)]};
    target[0] += F[p] * o->w;
    for (int d = 0; d < 3; ++d) target[1 + d] += v[d] * F[p] * o->w;
    target[4] += 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) * F[p] * o->w;
  }
  int polish = 0;
  for (int it = 1; it <= 50; ++it) {
    double R[5] = {0, 0, 0, 0, 0}, J[5][5];
    memset(J, 0, sizeof(J));
    double u[3] = {x[1], x[2], x[3]}, T = x[4];
    for (int p = 0; p < o->nvel; ++p) {
      double v[3] = {o->v[p % N], o->v[(p / N) % N], o->v[p / (N * N)]};
      double c[3] = {v[0] - u[0], v[1] - u[1], v[2] - u[2]};
      double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
      double M = maxw3(x[0], u, T, v[0], v[1], v[2]);
      double dM[5] = {M / x[0], M * c[0] / T, M * c[1] / T, M * c[2] / T,
                      M * (c2 / (2.0 * T * T) - 1.5 / T)};
      double psi[5] = {1.0, v[0], v[1], v[2], 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2])};
      for (int i = 0; i < 5; ++i) {
        R[i] += psi[i] * M * o->w;
        for (int j = 0; j < 5; ++j) J[i][j] += psi[i] * dM[j] * o->w;
      }
    }
    for (int i = 0; i < 5; ++i) R[i] -= target[i];
    if (solve5(5, J, R)) return -1;
    for (int i = 0; i < 5; ++i) x[i] -= R[i];
    if (polish) return it;
    double su = sqrt(fabs(x[4]));
    if (fabs(R[0]) <= 1e-13 * fabs(x[0]) && fabs(R[1]) <= 1e-13 * su && fabs(R[2]) <= 1e-13 * su &&
        fabs(R[3]) <= 1e-13 * su && fabs(R[4]) <= 1e-13 * fabs(x[4]))
      polish = 1;
  }
  return -1;
}

static int equilibrium3(const orc3d *o, const double *F, double *rho, double *u, double *T) {
  moments3(o, F, rho, u, T);
  if (!o->cfg.maxwellian) return 0;
  double x[5] = {*rho, u[0], u[1], u[2], *T};
  int it = conservative_triplet3(o, F, x);
  /* READING: a cell whose iteration does not converge keeps the direct triplet */
  if (it > 0) { *rho = x[0]; u[0] = x[1]; u[1] = x[2]; u[2] = x[3]; *T = x[4]; }
  return it;
}

int orc3d_equilibrium(const orc3d *o, const double *F, double *out) {
  double u[3];
  int it = equilibrium3(o, F, &out[0], u, &out[4]);
  out[1] = u[0]; out[2] = u[1]; out[3] = u[2];
  return it;
}

/* What the relaxation of one cell relaxes toward: the triplet and, for the
   Shakhov model, the heat flux q of eq. (MacroscopicTD), taken about the
   directly computed mean velocity (READING, as in 2D). */
typedef struct { double rho, u[3], T, q[3]; } relax3;

static void relax_target3(const orc3d *o, const double *F, relax3 *t) {
  equilibrium3(o, F, &t->rho, t->u, &t->T);
  t->q[0] = t->q[1] = t->q[2] = 0.0;
  if (o->cfg.model != 1) return;
  int N = o->N;
  double r, u[3], T;
  moments3(o, F, &r, u, &T);
  for (int p = 0; p < o->nvel; ++p) {
    double c[3] = {o->v[p % N] - u[0], o->v[(p / N) % N] - u[1], o->v[p / (N * N)] - u[2]};
    double h = 0.5 * (c[0] * c[0] + c[1] * c[1] + c[2] * c[2]) * F[p] * o->w;
    for (int d = 0; d < 3; ++d) t->q[d] += c[d] * h;
  }
}

/* equilibrium at v: the Maxwellian (BGK) or the Shakhov function of Section
   2.1, M [1 + (1 - Pr) (v - u).q (|v - u|^2/(R T) - 5) / (5 P R T)],
   P = rho R T, R = 1 */
static double equilibrium_at3(const orc3d *o, const relax3 *t, double vx, double vy, double vz) {
  double M = maxw3(t->rho, t->u, t->T, vx, vy, vz);
  if (o->cfg.model != 1) return M;
  double c[3] = {vx - t->u[0], vy - t->u[1], vz - t->u[2]};
  double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
  double cq = c[0] * t->q[0] + c[1] * t->q[1] + c[2] * t->q[2];
  double P = t->rho * t->T;
  return M * (1.0 + (1.0 - o->cfg.prandtl) * cq * (c2 / t->T - 5.0) / (5.0 * P * t->T));
}

void orc3d_equilibrium_values(const orc3d *o, const double *F, double *Fe) {
  relax3 t;
  relax_target3(o, F, &t);
  int N = o->N;
  for (int p = 0; p < o->nvel; ++p)
    Fe[p] = equilibrium_at3(o, &t, o->v[p % N], o->v[(p / N) % N], o->v[p / (N * N)]);
}

/* scheme (eq-schema3D) for control volume m, fixed geometry */
/* Update of one control volume from its transport residual R (the sum of
   its members' face and wall fluxes, velocity by velocity) and volume V:
   the explicit scheme with the relaxation of eq. (eq-schema3D), or the
   semi-implicit scheme (ImpSchemeDD in 3D). */
static void relax_update3(const orc3d *o, const double *fc, const double *R, double V, double *out) {
  int nvel = o->nvel, N = o->N;
  /* READING: conservative equilibrium -> the whole triplet, rho in tau
     included, from the Newton solution */
  relax3 tg;
  relax_target3(o, fc, &tg);
  double rho = tg.rho;
  int collide = o->cfg.kn > 0.0;
  double tau = collide ? sqrt(M_PI) / 2.0 * (1.0 / rho) * o->cfg.kn * o->cfg.lref / sqrt(2.0) : 1.0;
  if (o->cfg.scheme == 1) {
    /* semi-implicit scheme (ImpSchemeDD in 3D): equilibrium of the
       transported value, tau^n from the direct density at t^n (READING) */
    double *fs = calloc(nvel, sizeof(double));
    for (int p = 0; p < nvel; ++p) fs[p] = fc[p] - o->dt / V * R[p];
    double rn, un[3], Tn;
    moments3(o, fc, &rn, un, &Tn);
    double nu = collide ? o->dt / (sqrt(M_PI) / 2.0 * (1.0 / rn) * o->cfg.kn * o->cfg.lref / sqrt(2.0)) : 0.0;
    relax3 t1;
    relax_target3(o, fs, &t1);
    for (int p = 0; p < nvel; ++p) {
      double E = collide ? equilibrium_at3(o, &t1, o->v[p % N], o->v[(p / N) % N], o->v[p / (N * N)]) : 0.0;
      out[p] = (fs[p] + nu * E) / (1.0 + nu);
    }
    free(fs);
    return;
  }
  for (int p = 0; p < nvel; ++p) {
    double E = collide ? equilibrium_at3(o, &tg, o->v[p % N], o->v[(p / N) % N], o->v[p / (N * N)]) : 0.0;
    double fnew = fc[p] - o->dt / V * R[p];
    if (collide) fnew += o->dt / tau * (E - fc[p]);
    out[p] = fnew;
  }
}

/* Diffuse wall of zero net mass flux (Section 5 step 4), fixed wall
   u_w = 0, normal nwk into the solid: fw = phi_w M[1, 0, T_w] at every
   velocity, phi_w from the outgoing flux of the control-volume value fc. */
static void wall_values3(const orc3d *o, const double *fc, const double *nwk, double *fw) {
  int nvel = o->nvel, N = o->N;
  double Tw = o->cfg.t_wall, zero[3] = {0, 0, 0};
  double num = 0.0, den = 0.0;
  for (int p = 0; p < nvel; ++p) {
    double vx = o->v[p % N], vy = o->v[(p / N) % N], vz = o->v[p / (N * N)];
    double cn = vx * nwk[0] + vy * nwk[1] + vz * nwk[2];
    if (cn > 0.0) num += cn * fc[p] * o->w;
    else if (cn < 0.0) den += cn * maxw3(1.0, zero, Tw, vx, vy, vz) * o->w;
  }
  double phi = den != 0.0 ? -num / den : 0.0;
  for (int p = 0; p < nvel; ++p)
    fw[p] = phi * maxw3(1.0, zero, Tw, o->v[p % N], o->v[(p / N) % N], o->v[p / (N * N)]);
}

static void scheme3(const orc3d *o, const double *Fm, int m, double *out) {
  int nvel = o->nvel, N = o->N, nx = o->nx, ny = o->ny, nz = o->nz;
  const double *fc = Fm + (size_t)m * nvel;
  const double *in = o->cfg.inflow;
  double uin[3] = {in[1], in[2], in[3]};
  double *R = calloc(nvel, sizeof(double));
  double *fw = malloc(nvel * sizeof(double));
  for (int q = o->mptr[m]; q < o->mptr[m + 1]; ++q) {
    int k = o->midx[q];
    int i = k % nx, j = (k / nx) % ny, kk = k / (nx * ny);
    const double *fk = Fm + (size_t)k * nvel;
    int nb[6] = {i > 0 ? k - 1 : -1, i + 1 < nx ? k + 1 : -1, j > 0 ? k - nx : -1,
                 j + 1 < ny ? k + nx : -1, kk > 0 ? k - nx * ny : -1, kk + 1 < nz ? k + nx * ny : -1};
    int has_wall = o->sw[k] > 0.0;
    if (has_wall) {
      const double nwk[3] = {o->nw[0][k], o->nw[1][k], o->nw[2][k]};
      wall_values3(o, fc, nwk, fw);
    }
    for (int p = 0; p < nvel; ++p) {
      double vv[3] = {o->v[p % N], o->v[(p / N) % N], o->v[p / (N * N)]};
      double r = 0.0;
      for (int f = 0; f < 6; ++f) {
        double A = o->S[f][k];
        if (A == 0.0) continue;
        /* outward normal velocity of face f */
        double c = (f & 1) ? vv[f / 2] : -vv[f / 2];
        double fn = nb[f] >= 0 ? Fm[(size_t)nb[f] * nvel + p] : maxw3(in[0], uin, in[4], vv[0], vv[1], vv[2]);
        r += A * (mx(c, 0.0) * fk[p] + mn(c, 0.0) * fn);
      }
      if (has_wall) {
        double cn = vv[0] * o->nw[0][k] + vv[1] * o->nw[1][k] + vv[2] * o->nw[2][k];
        r += o->sw[k] * (mn(cn, 0.0) * fw[p] + mx(cn, 0.0) * fk[p]);
      }
      R[p] += r;
    }
  }
  relax_update3(o, fc, R, o->vcv[m], out);
  free(R); free(fw);
}

/* wall stress of one wall face (normal nwk into the solid, area swk) from
   the control-volume value fc, added to the force F (Section 5 step 5) */
static void wall_force3(const orc3d *o, const double *fc, const double *nwk, double swk, double *F) {
  int nvel = o->nvel, N = o->N;
  double Tw = o->cfg.t_wall, zero[3] = {0, 0, 0};
  double num = 0.0, den = 0.0;
  for (int p = 0; p < nvel; ++p) {
    double vx = o->v[p % N], vy = o->v[(p / N) % N], vz = o->v[p / (N * N)];
    double cn = vx * nwk[0] + vy * nwk[1] + vz * nwk[2];
    if (cn > 0.0) num += cn * fc[p] * o->w;
    else if (cn < 0.0) den += cn * maxw3(1.0, zero, Tw, vx, vy, vz) * o->w;
  }
  double phi = den != 0.0 ? -num / den : 0.0;
  double s[3] = {0, 0, 0};
  for (int p = 0; p < nvel; ++p) {
    double vv[3] = {o->v[p % N], o->v[(p / N) % N], o->v[p / (N * N)]};
    double cn = vv[0] * nwk[0] + vv[1] * nwk[1] + vv[2] * nwk[2];
    double fv = cn < 0.0 ? phi * maxw3(1.0, zero, Tw, vv[0], vv[1], vv[2]) : (cn > 0.0 ? fc[p] : 0.0);
    for (int d = 0; d < 3; ++d) s[d] += vv[d] * cn * fv * o->w;
  }
  for (int d = 0; d < 3; ++d) F[d] += s[d] * swk;
}

static void force3(const orc3d *o, const double *Fm, double *diag) {
  int nvel = o->nvel;
  double F[3] = {0, 0, 0}, mass = 0.0;
  for (int k = 0; k < o->ncell; ++k) {
    if (o->sw[k] <= 0.0) continue;
    const double nwk[3] = {o->nw[0][k], o->nw[1][k], o->nw[2][k]};
    wall_force3(o, Fm + (size_t)o->master[k] * nvel, nwk, o->sw[k], F);
  }
  for (int m = 0; m < o->ncell; ++m) {
    if (o->master[m] != m) continue;
    double sm = 0.0;
    for (int p = 0; p < nvel; ++p) sm += Fm[(size_t)m * nvel + p] * o->w;
    mass += o->vcv[m] * sm;
  }
  diag[0] = F[0]; diag[1] = F[1]; diag[2] = F[2]; diag[3] = mass;
}

void orc3d_force(const orc3d *o, const double *Fm, double *diag) { force3(o, Fm, diag); }

void orc3d_update_cells(const orc3d *o, const double *Fm, const int *cells, int ncells, double *out) {
  int nvel = o->nvel;
#pragma omp parallel for schedule(dynamic, 4)
  for (int q = 0; q < ncells; ++q) {
    int m = o->master[cells[q]];
    double *dst = out + (size_t)q * nvel;
    if (m < 0) { memset(dst, 0, nvel * sizeof(double)); continue; }
    scheme3(o, Fm, m, dst);
  }
}

int orc3d_step(orc3d *o, const double *F, double *Fo, double *diag) {
  int nvel = o->nvel;
  size_t tot = (size_t)o->ncell * nvel;
  double *Fm = malloc(tot * sizeof(double));
  memcpy(Fm, F, tot * sizeof(double));
  merge3(o, Fm);
  if (diag) force3(o, Fm, diag);
#pragma omp parallel for schedule(dynamic, 16)
  for (int m = 0; m < o->ncell; ++m) {
    if (o->master[m] != m) continue;
    scheme3(o, Fm, m, Fo + (size_t)m * nvel);
  }
  for (int c = 0; c < o->ncell; ++c) {
    int m = o->master[c];
    if (m < 0) memset(Fo + (size_t)c * nvel, 0, nvel * sizeof(double));
    else if (m != c) memcpy(Fo + (size_t)c * nvel, Fo + (size_t)m * nvel, nvel * sizeof(double));
  }
  free(Fm);
  return 0;
}

/* moments per cell, eq. (MacroscopicTD): rho, ux, uy, uz, T, Sxx, Sxy, Sxz,
   Syy, Syz, Szz, qx, qy, qz (14 per cell) */
void orc3d_moments(const orc3d *o, const double *F, double *out) {
  int N = o->N;
  for (int c = 0; c < o->ncell; ++c) {
    double *q = out + (size_t)c * 14;
    if (o->type[c] == SOLID) { for (int k = 0; k < 14; ++k) q[k] = 0.0; continue; }
    const double *fc = F + (size_t)c * o->nvel;
    double rho, u[3], T;
    moments3(o, fc, &rho, u, &T);
    double S[6] = {0, 0, 0, 0, 0, 0}, h[3] = {0, 0, 0};
    for (int p = 0; p < o->nvel; ++p) {
      double cx = o->v[p % N] - u[0], cy = o->v[(p / N) % N] - u[1], cz = o->v[p / (N * N)] - u[2];
      double fw = fc[p] * o->w;
      S[0] += cx * cx * fw; S[1] += cx * cy * fw; S[2] += cx * cz * fw;
      S[3] += cy * cy * fw; S[4] += cy * cz * fw; S[5] += cz * cz * fw;
      double e = 0.5 * (cx * cx + cy * cy + cz * cz) * fw;
      h[0] += cx * e; h[1] += cy * e; h[2] += cz * e;
    }
    q[0] = rho; q[1] = u[0]; q[2] = u[1]; q[3] = u[2]; q[4] = T;
    for (int k = 0; k < 6; ++k) q[5 + k] = S[k];
    for (int k = 0; k < 3; ++k) q[11 + k] = h[k];
  }
}

void orc3d_velocity(const orc3d *o, double *v) { memcpy(v, o->v, o->N * sizeof(double)); }

/* ================================================================== */
/* Octree mesh (Section 5.1, octree procedure) around a fixed body        */
/* ================================================================== */
/* The coarse n[0] x n[1] x n[2] grid is refined near the boundary: a cell
   of depth d is divided in 8 when its centre is closer to the boundary than
   band * Delta x / 2^d and d < amr_depth.  READINGS: the distance is the
   absolute value of the level set at the centre; Delta x is the largest
   coarse spacing; "d <= d_max" is read as "a cell of depth d < d_max is
   divided", so the finest depth is d_max (the paper's 50^3 coarse grid with
   d_max = 2 then has the resolution of a 200^3 grid near the vanes); band =
   2 sqrt 2 unless amr_band > 0.  The data structure: leaves in Z-order of
   their lower corner (in finest-level units), and per leaf a list of faces
   in the order x-, x+, y-, y+, z-, z+: the leaf across (same depth, one
   coarser, or the four of the next finer depth) or the farfield (-1), with
   the face's gas area.  Cut cells lie at the finest depth (the band is
   wider than a cell's half-diagonal) and have the uniform grid's geometry
   there; their control volumes follow the same master search, restricted to
   leaves of the finest depth.

   Rotating body (Section 5, steps 1-7, pure rotation about the z axis
   through the body centre): a step on the mesh of t^n, then the mesh is
   rebuilt for the body at t^{n+1} (the adaptation the paper makes at the
   start of the next iteration) and the state is carried over by
   restriction (gas-volume weighted mean of the old leaves inside a new one)
   or prolongation (a new leaf inside an old one takes its value). */
typedef unsigned long long u64;
typedef struct { u64 key; int idx; } keyidx3;

struct orc3a {
  orc_cfg cfg;
  orc3d vel;                      /* velocity grid, model and dt (helpers shared with orc3d) */
  int n0[3], dmax, nleaf, nface;
  double hf[3];                   /* finest spacing */
  double th, om;                  /* body angle about z and angular velocity */
  int *lvl, *ijk;                 /* depth and integer coordinates at that depth (3 per leaf) */
  int *type, *master, *mptr, *midx;
  int *fptr, *fnb, *fdir;
  double *farea;
  double *S6;                     /* 6 gas face areas per leaf */
  double *vsum;                   /* sum of the 8 vertex values (centre test) */
  double *sw, *nw3, *rw3, *vbar, *vcv;
  keyidx3 *tab;                   /* (depth, coordinates) -> leaf, sorted by key */
  double *vbar1;                  /* leaves' gas volumes with the body at t^{n+1} (last step) */
  int pn, *plvl, *pijk;           /* previous mesh, kept by orc3a_adapt for orc3a_remap */
  double *pvbar;                  /* its leaves' gas volumes at the new angle */
  keyidx3 *ptab;
};

static u64 cell_key3(int l, int i, int j, int k) {
  return ((u64)l << 60) | ((u64)i << 40) | ((u64)j << 20) | (u64)k;
}

static u64 spread3(u64 x) {
  u64 r = 0;
  for (int b = 0; b < 21; ++b) r |= ((x >> b) & 1ULL) << (3 * b);
  return r;
}

static int cmp_keyidx3(const void *a, const void *b) {
  u64 x = ((const keyidx3 *)a)->key, y = ((const keyidx3 *)b)->key;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* leaf with this (depth, coordinates), or -1 */
static int find_leaf3(const keyidx3 *tab, int n, int l, int i, int j, int k) {
  if (l < 0 || i < 0 || j < 0 || k < 0) return -1;
  u64 key = cell_key3(l, i, j, k);
  int lo = 0, hi = n - 1;
  while (lo <= hi) {
    int mid = (lo + hi) / 2;
    if (tab[mid].key == key) return tab[mid].idx;
    if (tab[mid].key < key) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

void orc3a_destroy(orc3a *o);

/* geometry of leaf q with the body at angle th: the 8 vertex values clamped
   as on the uniform grid, then the uniform grid's per-cell construction at
   the leaf's own size.  Returns 1 for a saddle face. */
static int leaf_geom3a(const orc3a *o, double th, int q, int *type, double *S6, double *sw, double *nw,
                       double *rw, double *vbar, double *vsum) {
  const orc_cfg *cf = &o->cfg;
  int l = o->lvl[q], sh = o->dmax - l;
  int A0[3] = {o->ijk[3 * q] << sh, o->ijk[3 * q + 1] << sh, o->ijk[3 * q + 2] << sh};
  double q8[8], h[3], eps = 1e-10 * o->hf[0];
  for (int d = 0; d < 3; ++d) h[d] = o->hf[d] * (double)(1 << sh);
  for (int t = 0; t < 8; ++t) {
    int a = A0[0] + ((t & 1) << sh), b = A0[1] + (((t >> 1) & 1) << sh), c = A0[2] + (((t >> 2) & 1) << sh);
    double p = levelset3(cf, th, cf->lo[0] + a * o->hf[0], cf->lo[1] + b * o->hf[1], cf->lo[2] + c * o->hf[2]);
    double sg = p >= 0.0 ? 1.0 : -1.0;
    q8[t] = sg * mx(fabs(p), eps);
  }
  double vs = 0.0;
  for (int t = 0; t < 8; ++t) vs += q8[t];
  *vsum = vs;
  double rl[3];
  int bad = cell_geom3(q8, h, type, S6, sw, nw, rl, vbar);
  for (int d = 0; d < 3; ++d) rw[d] = *sw > 0.0 ? cf->lo[d] + A0[d] * o->hf[d] + rl[d] : 0.0;
  return bad;
}

static void free_mesh3a(orc3a *o) {
  free(o->lvl); free(o->ijk); free(o->type); free(o->master); free(o->mptr); free(o->midx);
  free(o->fptr); free(o->fnb); free(o->fdir); free(o->farea); free(o->S6); free(o->vsum);
  free(o->sw); free(o->nw3); free(o->rw3); free(o->vbar); free(o->vcv); free(o->tab); free(o->vbar1);
  o->lvl = o->ijk = o->type = o->master = o->mptr = o->midx = o->fptr = o->fnb = o->fdir = NULL;
  o->farea = o->S6 = o->vsum = o->sw = o->nw3 = o->rw3 = o->vbar = o->vcv = o->vbar1 = NULL;
  o->tab = NULL;
}

/* the mesh for the body at angle o->th */
static int build3a(orc3a *o) {
  const orc_cfg *cf = &o->cfg;
  int D = o->dmax;
  double h0[3];
  for (int d = 0; d < 3; ++d) h0[d] = (cf->hi[d] - cf->lo[d]) / o->n0[d];
  double Dx = mx(h0[0], mx(h0[1], h0[2]));
  double band = cf->amr_band > 0.0 ? cf->amr_band : 2.0 * sqrt(2.0);
  /* refinement by the criterion, depth first */
  int cap = 1 << 16, nl = 0, sp = 0, scap = 1 << 12;
  int *leaf = malloc((size_t)cap * 4 * sizeof(int));
  int *st = malloc((size_t)scap * 4 * sizeof(int));
  for (int k = o->n0[2] - 1; k >= 0; --k)
    for (int j = o->n0[1] - 1; j >= 0; --j)
      for (int i = o->n0[0] - 1; i >= 0; --i) {
        if (sp == scap) { scap *= 2; st = realloc(st, (size_t)scap * 4 * sizeof(int)); }
        st[4 * sp] = 0; st[4 * sp + 1] = i; st[4 * sp + 2] = j; st[4 * sp + 3] = k; ++sp;
      }
  while (sp > 0) {
    --sp;
    int l = st[4 * sp], i = st[4 * sp + 1], j = st[4 * sp + 2], k = st[4 * sp + 3];
    double s = 1.0 / (double)(1 << l);
    double cx = cf->lo[0] + (i + 0.5) * h0[0] * s, cy = cf->lo[1] + (j + 0.5) * h0[1] * s,
           cz = cf->lo[2] + (k + 0.5) * h0[2] * s;
    if (l < D && fabs(levelset3(cf, o->th, cx, cy, cz)) < band * Dx * s) {
      for (int t = 7; t >= 0; --t) {
        if (sp == scap) { scap *= 2; st = realloc(st, (size_t)scap * 4 * sizeof(int)); }
        st[4 * sp] = l + 1;
        st[4 * sp + 1] = 2 * i + (t & 1); st[4 * sp + 2] = 2 * j + ((t >> 1) & 1);
        st[4 * sp + 3] = 2 * k + ((t >> 2) & 1);
        ++sp;
      }
    } else {
      if (nl == cap) { cap *= 2; leaf = realloc(leaf, (size_t)cap * 4 * sizeof(int)); }
      memcpy(leaf + 4 * nl, st + 4 * sp, 4 * sizeof(int));
      ++nl;
    }
  }
  free(st);
  /* Z-order of the lower corner in finest units */
  keyidx3 *mz = malloc((size_t)nl * sizeof(keyidx3));
  for (int q = 0; q < nl; ++q) {
    int l = leaf[4 * q], sh = D - l;
    u64 I = (u64)leaf[4 * q + 1] << sh, J = (u64)leaf[4 * q + 2] << sh, K = (u64)leaf[4 * q + 3] << sh;
    mz[q].key = spread3(I) | (spread3(J) << 1) | (spread3(K) << 2);
    mz[q].idx = q;
  }
  qsort(mz, nl, sizeof(keyidx3), cmp_keyidx3);
  int n = o->nleaf = nl;
  o->lvl = malloc(n * sizeof(int)); o->ijk = malloc((size_t)n * 3 * sizeof(int));
  for (int q = 0; q < n; ++q) {
    const int *c = leaf + 4 * mz[q].idx;
    o->lvl[q] = c[0];
    o->ijk[3 * q] = c[1]; o->ijk[3 * q + 1] = c[2]; o->ijk[3 * q + 2] = c[3];
  }
  free(mz); free(leaf);
  keyidx3 *tab = o->tab = malloc((size_t)n * sizeof(keyidx3));
  for (int q = 0; q < n; ++q) {
    tab[q].key = cell_key3(o->lvl[q], o->ijk[3 * q], o->ijk[3 * q + 1], o->ijk[3 * q + 2]);
    tab[q].idx = q;
  }
  qsort(tab, n, sizeof(keyidx3), cmp_keyidx3);
  o->type = calloc(n, sizeof(int)); o->master = calloc(n, sizeof(int));
  o->mptr = calloc(n + 1, sizeof(int)); o->midx = calloc(n, sizeof(int));
  o->S6 = calloc((size_t)n * 6, sizeof(double)); o->vsum = calloc(n, sizeof(double));
  o->sw = calloc(n, sizeof(double)); o->nw3 = calloc((size_t)n * 3, sizeof(double));
  o->rw3 = calloc((size_t)n * 3, sizeof(double));
  o->vbar = calloc(n, sizeof(double)); o->vcv = calloc(n, sizeof(double));
  int bad = 0;
  for (int q = 0; q < n; ++q) {
    int type;
    if (leaf_geom3a(o, o->th, q, &type, o->S6 + 6 * q, &o->sw[q], o->nw3 + 3 * q, o->rw3 + 3 * q, &o->vbar[q],
                    &o->vsum[q]))
      bad = 1;
    if (type == CUT && o->lvl[q] < D) bad = 1;     /* a cut cell above the finest depth */
    o->type[q] = type;
  }
  /* faces */
  int fcap = 8 * n + 16;
  o->fptr = calloc(n + 1, sizeof(int));
  o->fnb = malloc((size_t)fcap * sizeof(int)); o->fdir = malloc((size_t)fcap * sizeof(int));
  o->farea = malloc((size_t)fcap * sizeof(double));
  int nf = 0;
#define ADDF(nb_, t_, a_) do { if (nf == fcap) { fcap *= 2; \
    o->fnb = realloc(o->fnb, (size_t)fcap * sizeof(int)); o->fdir = realloc(o->fdir, (size_t)fcap * sizeof(int)); \
    o->farea = realloc(o->farea, (size_t)fcap * sizeof(double)); } \
    o->fnb[nf] = (nb_); o->fdir[nf] = (t_); o->farea[nf] = (a_); ++nf; } while (0)
  for (int q = 0; q < n; ++q) {
    o->fptr[q] = nf;
    if (o->type[q] == SOLID) continue;
    int l = o->lvl[q];
    for (int t = 0; t < 6; ++t) {
      double A = o->S6[6 * q + t];
      if (A == 0.0) continue;
      int d = t >> 1, sd = t & 1, d1 = (d + 1) % 3, d2 = (d + 2) % 3;
      int g[3] = {o->ijk[3 * q], o->ijk[3 * q + 1], o->ijk[3 * q + 2]};
      g[d] += sd ? 1 : -1;
      if (g[d] < 0 || g[d] >= (o->n0[d] << l)) { ADDF(-1, t, A); continue; }
      int x = find_leaf3(tab, n, l, g[0], g[1], g[2]);
      if (x < 0) x = find_leaf3(tab, n, l - 1, g[0] >> 1, g[1] >> 1, g[2] >> 1);
      if (x >= 0) { ADDF(x, t, A); continue; }
      if (l == D) { bad = 1; continue; }
      for (int b2 = 0; b2 < 2; ++b2)
        for (int b1 = 0; b1 < 2; ++b1) {
          int c[3];
          c[d] = 2 * g[d] + (sd ? 0 : 1); c[d1] = 2 * g[d1] + b1; c[d2] = 2 * g[d2] + b2;
          int y = find_leaf3(tab, n, l + 1, c[0], c[1], c[2]);
          if (y < 0) { bad = 1; continue; }          /* more than one depth apart */
          double Ay = o->S6[6 * y + (t ^ 1)];         /* the finer leaf's face toward this one */
          if (Ay != 0.0) ADDF(y, t, Ay);
        }
    }
  }
  o->fptr[n] = nf;
  o->nface = nf;
#undef ADDF
  /* masters (finest depth): centre in gas = mean of the 8 vertex values
     > 1e-12 dx; hop across the largest face shared with a leaf of the same
     depth, order x+, x-, y+, y-, z+, z- */
  double thr = 1e-12 * o->hf[0];
  const int order[6] = {1, 0, 3, 2, 5, 4};
  for (int q = 0; q < n; ++q) {
    if (o->type[q] == SOLID) { o->master[q] = -1; continue; }
    int cur = q, hops = 0, seen[5];
    seen[0] = q;
    for (;;) {
      if (o->vsum[cur] / 8.0 > thr) break;
      int l = o->lvl[cur], nb6[6];
      double L[6];
      for (int u = 0; u < 6; ++u) {
        int t = order[u], d = t >> 1;
        int g[3] = {o->ijk[3 * cur], o->ijk[3 * cur + 1], o->ijk[3 * cur + 2]};
        g[d] += (t & 1) ? 1 : -1;
        nb6[u] = -1;
        L[u] = 0.0;
        if (g[d] < 0 || g[d] >= (o->n0[d] << l)) continue;
        nb6[u] = find_leaf3(tab, n, l, g[0], g[1], g[2]);
        L[u] = o->S6[6 * cur + t];
      }
      double M = 0.0;
      for (int u = 0; u < 6; ++u) M = mx(M, L[u]);
      if (!(M > 0.0) || hops == 4) { bad = 1; break; }
      double tie = M * (1.0 - 1e-12);
      int u = 0;
      while (L[u] < tie) ++u;
      if (nb6[u] < 0) { bad = 1; break; }       /* across a change of depth */
      cur = nb6[u];
      ++hops;
      for (int hh = 0; hh < hops; ++hh) if (seen[hh] == cur) bad = 1;
      if (bad) break;
      seen[hops] = cur;
    }
    o->master[q] = cur;
  }
  if (bad) return -3;
  memset(o->mptr, 0, (n + 1) * sizeof(int));
  for (int c = 0; c < n; ++c) if (o->master[c] >= 0) o->mptr[o->master[c] + 1]++;
  for (int c = 0; c < n; ++c) o->mptr[c + 1] += o->mptr[c];
  int *fill = calloc(n, sizeof(int));
  for (int c = 0; c < n; ++c) {
    int m = o->master[c];
    if (m >= 0) o->midx[o->mptr[m] + fill[m]++] = c;
  }
  free(fill);
  for (int c = 0; c < n; ++c) {
    o->vcv[c] = 0.0;
    for (int q = o->mptr[c]; q < o->mptr[c + 1]; ++q) o->vcv[c] += o->vbar[o->midx[q]];
  }
  for (int c = 0; c < n; ++c) {
    int m = o->master[c];
    if (m >= 0 && o->master[m] != m) return -3;
  }
  return 0;
}

int orc3a_create(const orc_cfg *cfg, orc3a **out) {
  if (!cfg || cfg->dim != 3 || cfg->n[0] < 1 || cfg->n[1] < 1 || cfg->n[2] < 1 || cfg->nv < 1 ||
      !(cfg->vmax > cfg->vmin) || cfg->amr_depth < 0 || cfg->amr_depth > 8)
    return -1;
  if (cfg->motion != 0 && cfg->body_kind != 0 && cfg->motion == 1 && !(cfg->inertia > 0.0)) return -1;
  for (int d = 0; d < 3; ++d)
    if (((u64)cfg->n[d] << cfg->amr_depth) >= (1ULL << 20)) return -1;
  orc3a *o = calloc(1, sizeof(orc3a));
  o->cfg = *cfg;
  o->dmax = cfg->amr_depth;
  o->th = cfg->theta;
  o->om = cfg->motion != 0 ? cfg->omega : 0.0;
  for (int d = 0; d < 3; ++d) {
    o->n0[d] = cfg->n[d];
    o->hf[d] = (cfg->hi[d] - cfg->lo[d]) / (double)(cfg->n[d] << o->dmax);
  }
  /* velocity grid, model and time step: the finest spacing sets dt */
  orc3d *v = &o->vel;
  v->cfg = *cfg;
  v->N = cfg->nv; v->nvel = v->N * v->N * v->N;
  v->dx = o->hf[0]; v->dy = o->hf[1]; v->dz = o->hf[2];
  v->dv = (cfg->vmax - cfg->vmin) / v->N;
  v->w = v->dv * v->dv * v->dv;
  v->v = malloc(v->N * sizeof(double));
  for (int p = 0; p < v->N; ++p) v->v[p] = cfg->vmin + (p + 0.5) * v->dv;
  double vm = 0.0;
  for (int p = 0; p < v->N; ++p) vm = mx(vm, fabs(v->v[p]));
  v->dt = cfg->dt > 0.0 ? cfg->dt : cfg->cfl / (vm / v->dx + vm / v->dy + vm / v->dz);
  int st = build3a(o);
  if (st) { orc3a_destroy(o); return st; }
  *out = o;
  return 0;
}

void orc3a_destroy(orc3a *o) {
  if (!o) return;
  free(o->vel.v);
  free_mesh3a(o);
  free(o->plvl); free(o->pijk); free(o->pvbar); free(o->ptab);
  free(o);
}

double orc3a_dt(const orc3a *o) { return o->vel.dt; }
int orc3a_nleaf(const orc3a *o) { return o->nleaf; }
int orc3a_nface(const orc3a *o) { return o->nface; }
void orc3a_velocity(const orc3a *o, double *v) { memcpy(v, o->vel.v, o->vel.N * sizeof(double)); }
void orc3a_body(const orc3a *o, double *out) { out[0] = o->th; out[1] = o->om; }

void orc3a_leaves(const orc3a *o, int *lvl, int *ijk, int *type, int *master, double *vbar,
                  double *vcv, double *sw, double *S6) {
  int n = o->nleaf;
  memcpy(lvl, o->lvl, n * sizeof(int));
  memcpy(ijk, o->ijk, (size_t)n * 3 * sizeof(int));
  memcpy(type, o->type, n * sizeof(int));
  memcpy(master, o->master, n * sizeof(int));
  memcpy(vbar, o->vbar, n * sizeof(double));
  memcpy(vcv, o->vcv, n * sizeof(double));
  memcpy(sw, o->sw, n * sizeof(double));
  memcpy(S6, o->S6, (size_t)n * 6 * sizeof(double));
}

void orc3a_faces(const orc3a *o, int *fptr, int *fnb, int *fdir, double *farea) {
  memcpy(fptr, o->fptr, (o->nleaf + 1) * sizeof(int));
  memcpy(fnb, o->fnb, o->nface * sizeof(int));
  memcpy(fdir, o->fdir, o->nface * sizeof(int));
  memcpy(farea, o->farea, o->nface * sizeof(double));
}

void orc3a_init(const orc3a *o, double *F) {
  const double *in = o->cfg.inflow;
  double u[3] = {in[1], in[2], in[3]};
  const orc3d *v = &o->vel;
  int N = v->N, nvel = v->nvel;
  for (int c = 0; c < o->nleaf; ++c)
    for (int p = 0; p < nvel; ++p) {
      double M = maxw3(in[0], u, in[4], v->v[p % N], v->v[(p / N) % N], v->v[p / (N * N)]);
      F[(size_t)c * nvel + p] = o->type[c] == SOLID ? 0.0 : M;
    }
}

static void merge3a(const orc3a *o, double *F) {
  int nvel = o->vel.nvel;
  double *acc = malloc(nvel * sizeof(double));
  for (int m = 0; m < o->nleaf; ++m) {
    if (o->master[m] != m || o->mptr[m + 1] - o->mptr[m] <= 1) continue;
    for (int p = 0; p < nvel; ++p) acc[p] = 0.0;
    for (int q = o->mptr[m]; q < o->mptr[m + 1]; ++q) {
      int c = o->midx[q];
      for (int p = 0; p < nvel; ++p) acc[p] += o->vbar[c] * F[(size_t)c * nvel + p];
    }
    for (int q = o->mptr[m]; q < o->mptr[m + 1]; ++q) {
      int c = o->midx[q];
      for (int p = 0; p < nvel; ++p) F[(size_t)c * nvel + p] = acc[p] / o->vcv[m];
    }
  }
  free(acc);
}

void orc3a_merge(const orc3a *o, double *F) { merge3a(o, F); }

/* eq. (eq-schema3D) for the control volume of master m: the fluxes of its
   members' face lists and wall faces, then the update of the uniform grid */
static void scheme3a(const orc3a *o, const double *Fm, int m, double *out) {
  const orc3d *v = &o->vel;
  int nvel = v->nvel, N = v->N;
  const double *fc = Fm + (size_t)m * nvel;
  const double *in = o->cfg.inflow;
  double uin[3] = {in[1], in[2], in[3]};
  double *R = calloc(nvel, sizeof(double));
  double *fw = malloc(nvel * sizeof(double));
  for (int q = o->mptr[m]; q < o->mptr[m + 1]; ++q) {
    int k = o->midx[q];
    const double *fk = Fm + (size_t)k * nvel;
    int has_wall = o->sw[k] > 0.0;
    if (has_wall) wall_values3(v, fc, o->nw3 + 3 * k, fw);
    for (int p = 0; p < nvel; ++p) {
      double vv[3] = {v->v[p % N], v->v[(p / N) % N], v->v[p / (N * N)]};
      double r = 0.0;
      for (int e = o->fptr[k]; e < o->fptr[k + 1]; ++e) {
        double A = o->farea[e];
        int f = o->fdir[e];
        /* outward normal velocity of the face */
        double c = (f & 1) ? vv[f / 2] : -vv[f / 2];
        double fn = o->fnb[e] >= 0 ? Fm[(size_t)o->fnb[e] * nvel + p]
                                   : maxw3(in[0], uin, in[4], vv[0], vv[1], vv[2]);
        r += A * (mx(c, 0.0) * fk[p] + mn(c, 0.0) * fn);
      }
      if (has_wall) {
        const double *nk = o->nw3 + 3 * k;
        double cn = vv[0] * nk[0] + vv[1] * nk[1] + vv[2] * nk[2];
        r += o->sw[k] * (mn(cn, 0.0) * fw[p] + mx(cn, 0.0) * fk[p]);
      }
      R[p] += r;
    }
  }
  relax_update3(v, fc, R, o->vcv[m], out);
  free(R); free(fw);
}

/* ---- rotating body ---- */

/* velocity of the wall point r of a body turning at om about the z axis
   through its centre (step 4): om e_z x (r - centre).  READING: the printed
   r om (sin a, cos a, 0) is taken as this rigid rotation. */
static void wall_velocity3(const orc3a *o, const double *r, double om, double *uw) {
  uw[0] = -om * (r[1] - o->cfg.center[1]);
  uw[1] = om * (r[0] - o->cfg.center[0]);
  uw[2] = 0.0;
}

/* wall value of one wall face moving with uw (step 4): incoming and
   outgoing sets and the density from the relative velocity v - uw */
static void wall_values3m(const orc3d *o, const double *fc, const double *nwk, const double *uw, double *fw) {
  int nvel = o->nvel, N = o->N;
  double Tw = o->cfg.t_wall, num = 0.0, den = 0.0;
  for (int p = 0; p < nvel; ++p) {
    double vx = o->v[p % N], vy = o->v[(p / N) % N], vz = o->v[p / (N * N)];
    double cn = (vx - uw[0]) * nwk[0] + (vy - uw[1]) * nwk[1] + (vz - uw[2]) * nwk[2];
    if (cn > 0.0) num += cn * fc[p] * o->w;
    else if (cn < 0.0) den += cn * maxw3(1.0, uw, Tw, vx, vy, vz) * o->w;
  }
  double phi = den != 0.0 ? -num / den : 0.0;
  for (int p = 0; p < nvel; ++p)
    fw[p] = phi * maxw3(1.0, uw, Tw, o->v[p % N], o->v[(p / N) % N], o->v[p / (N * N)]);
}

/* force of one moving wall face (step 5): the relative-velocity stress
   (v - uw) ((v - uw).n) of the wall value on incoming and of the control
   volume's value on outgoing velocities, times the face area */
static void wall_force3m(const orc3d *o, const double *fc, const double *nwk, const double *uw, double swk,
                         double *Fk) {
  int nvel = o->nvel, N = o->N;
  double *fw = malloc(nvel * sizeof(double));
  wall_values3m(o, fc, nwk, uw, fw);
  double s[3] = {0, 0, 0};
  for (int p = 0; p < nvel; ++p) {
    double c[3] = {o->v[p % N] - uw[0], o->v[(p / N) % N] - uw[1], o->v[p / (N * N)] - uw[2]};
    double cn = c[0] * nwk[0] + c[1] * nwk[1] + c[2] * nwk[2];
    double fv = cn < 0.0 ? fw[p] : (cn > 0.0 ? fc[p] : 0.0);
    for (int d = 0; d < 3; ++d) s[d] += c[d] * cn * fv * o->w;
  }
  for (int d = 0; d < 3; ++d) Fk[d] = s[d] * swk;
  free(fw);
}

/* eq. (eq-schema3D) with the volume ratio V^n / V^{n+1,*} for the control
   volume of master m of t^n (vnew = its volume with the body at t^{n+1}),
   walls moving at om */
static void scheme3a_moving(const orc3a *o, const double *Fm, int m, double vnew, double om, double *out) {
  const orc3d *v = &o->vel;
  int nvel = v->nvel, N = v->N;
  const double *fc = Fm + (size_t)m * nvel;
  const double *in = o->cfg.inflow;
  double uin[3] = {in[1], in[2], in[3]};
  double *R = calloc(nvel, sizeof(double));
  double *fw = malloc(nvel * sizeof(double));
  for (int q = o->mptr[m]; q < o->mptr[m + 1]; ++q) {
    int k = o->midx[q];
    const double *fk = Fm + (size_t)k * nvel;
    int has_wall = o->sw[k] > 0.0;
    double uw[3] = {0, 0, 0};
    if (has_wall) {
      wall_velocity3(o, o->rw3 + 3 * k, om, uw);
      wall_values3m(v, fc, o->nw3 + 3 * k, uw, fw);
    }
    for (int p = 0; p < nvel; ++p) {
      double vv[3] = {v->v[p % N], v->v[(p / N) % N], v->v[p / (N * N)]};
      double r = 0.0;
      for (int e = o->fptr[k]; e < o->fptr[k + 1]; ++e) {
        double A = o->farea[e];
        int f = o->fdir[e];
        double c = (f & 1) ? vv[f / 2] : -vv[f / 2];
        double fn = o->fnb[e] >= 0 ? Fm[(size_t)o->fnb[e] * nvel + p]
                                   : maxw3(in[0], uin, in[4], vv[0], vv[1], vv[2]);
        r += A * (mx(c, 0.0) * fk[p] + mn(c, 0.0) * fn);
      }
      if (has_wall) {
        const double *nk = o->nw3 + 3 * k;
        double cn = (vv[0] - uw[0]) * nk[0] + (vv[1] - uw[1]) * nk[1] + (vv[2] - uw[2]) * nk[2];
        r += o->sw[k] * (mn(cn, 0.0) * fw[p] + mx(cn, 0.0) * fk[p]);
      }
      R[p] += r;
    }
  }
  relax3 tg;
  relax_target3(v, fc, &tg);
  int collide = o->cfg.kn > 0.0;
  double tau = collide ? sqrt(M_PI) / 2.0 * (1.0 / tg.rho) * o->cfg.kn * o->cfg.lref / sqrt(2.0) : 1.0;
  double ratio = o->vcv[m] / vnew;
  for (int p = 0; p < nvel; ++p) {
    double E = collide ? equilibrium_at3(v, &tg, v->v[p % N], v->v[(p / N) % N], v->v[p / (N * N)]) : 0.0;
    double fnew = ratio * fc[p] - v->dt / vnew * R[p];
    if (collide) fnew += ratio * (v->dt / tau) * (E - fc[p]);
    out[p] = fnew;
  }
  free(R); free(fw);
}

/* one step with the body turning (Section 5, steps 1-7) on the current
   mesh: Fo is the state at t^{n+1} on the same leaves, with the geometry of
   the body at t^{n+1}.  diag = Fx, Fy, torque about the z axis, mass of F^n. */
static int step3a_moving(orc3a *o, const double *F, double *Fo, double *diag) {
  const orc3d *v = &o->vel;
  int nvel = v->nvel, n = o->nleaf, D = o->dmax;
  size_t tot = (size_t)n * nvel;
  /* 1. angle at t^{n+1} (pure rotation, eq. motionDD_posit) */
  double th1 = o->th + v->dt * o->om;
  /* 2. merge over the control volumes of t^n */
  double *Fm = malloc(tot * sizeof(double));
  memcpy(Fm, F, tot * sizeof(double));
  merge3a(o, Fm);
  /* 3. the leaves with the body at t^{n+1}: types, gas volumes, faces */
  int *type1 = malloc(n * sizeof(int)), *target = malloc(n * sizeof(int));
  double *vbar1 = malloc(n * sizeof(double)), *S61 = malloc((size_t)n * 6 * sizeof(double));
  int bad = 0;
  for (int q = 0; q < n; ++q) {
    double sw1, nw1[3], rw1[3], vs1;
    if (leaf_geom3a(o, th1, q, &type1[q], S61 + 6 * q, &sw1, nw1, rw1, &vbar1[q], &vs1)) bad = 1;
    if (type1[q] == CUT && o->lvl[q] < D) bad = 1;   /* the body moved past the refined band */
    target[q] = o->master[q];
  }
  /* READING (as in 2D): a leaf solid at t^n and not at t^{n+1} joins the
     control volume of t^n reached by hopping across its largest face at
     t^{n+1} (same depth, order x+, x-, y+, y-, z+, z-, at most 4 hops) */
  const int order[6] = {1, 0, 3, 2, 5, 4};
  for (int q = 0; q < n && !bad; ++q) {
    if (!(o->type[q] == SOLID && type1[q] != SOLID)) continue;
    int cur = q, hops = 0;
    while (o->master[cur] < 0 && hops < 4) {
      int l = o->lvl[cur], nb = -1;
      double M = 0.0, L[6];
      int nb6[6];
      for (int u = 0; u < 6; ++u) {
        int t = order[u], d = t >> 1;
        int g[3] = {o->ijk[3 * cur], o->ijk[3 * cur + 1], o->ijk[3 * cur + 2]};
        g[d] += (t & 1) ? 1 : -1;
        nb6[u] = -1; L[u] = 0.0;
        if (g[d] < 0 || g[d] >= (o->n0[d] << l)) continue;
        nb6[u] = find_leaf3(o->tab, n, l, g[0], g[1], g[2]);
        L[u] = S61[6 * cur + t];
        M = mx(M, L[u]);
      }
      if (!(M > 0.0)) break;
      double tie = M * (1.0 - 1e-12);
      int u = 0;
      while (L[u] < tie) ++u;
      nb = nb6[u];
      if (nb < 0) break;
      cur = nb;
      ++hops;
    }
    if (o->master[cur] < 0) bad = 1;
    else target[q] = o->master[cur];
  }
  if (bad) { free(Fm); free(type1); free(target); free(vbar1); free(S61); return -3; }
  double *vnew = calloc(n, sizeof(double));
  for (int q = 0; q < n; ++q)
    if (target[q] >= 0) vnew[target[q]] += vbar1[q];
  /* 4-5. wall condition, force and torque at t^n */
  double Fw[3] = {0, 0, 0}, Tz = 0.0, mass = 0.0;
  for (int k = 0; k < n; ++k) {
    if (!(o->sw[k] > 0.0)) continue;
    double uw[3], Fk[3];
    wall_velocity3(o, o->rw3 + 3 * k, o->om, uw);
    wall_force3m(v, Fm + (size_t)o->master[k] * nvel, o->nw3 + 3 * k, uw, o->sw[k], Fk);
    for (int d = 0; d < 3; ++d) Fw[d] += Fk[d];
    Tz += (o->rw3[3 * k] - o->cfg.center[0]) * Fk[1] - (o->rw3[3 * k + 1] - o->cfg.center[1]) * Fk[0];
  }
  for (int m = 0; m < n; ++m) {
    if (o->master[m] != m) continue;
    double sm = 0.0;
    for (int p = 0; p < nvel; ++p) sm += Fm[(size_t)m * nvel + p] * v->w;
    mass += o->vcv[m] * sm;
  }
  if (diag) { diag[0] = Fw[0]; diag[1] = Fw[1]; diag[2] = Tz; diag[3] = mass; }
  /* 6. scheme on every control volume of t^n */
  double *Fcv = malloc(tot * sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
  for (int m = 0; m < n; ++m) {
    if (o->master[m] != m || !(vnew[m] > 0.0)) continue;
    scheme3a_moving(o, Fm, m, vnew[m], o->om, Fcv + (size_t)m * nvel);
  }
  /* 7. redistribution to the leaves of t^{n+1} */
  for (int q = 0; q < n; ++q) {
    int m = target[q];
    double *dst = Fo + (size_t)q * nvel;
    if (m < 0 || type1[q] == SOLID || !(vnew[m] > 0.0)) memset(dst, 0, nvel * sizeof(double));
    else memcpy(dst, Fcv + (size_t)m * nvel, nvel * sizeof(double));
  }
  /* body: explicit Euler, torque of t^n (free rotation) */
  if (o->cfg.motion == 1) o->om = o->om + v->dt * Tz / o->cfg.inertia;
  o->th = th1;
  free(o->vbar1);
  o->vbar1 = vbar1;
  free(Fm); free(Fcv); free(type1); free(target); free(S61); free(vnew);
  return 0;
}

/* one step on the octree; diag (nullable) = Fx, Fy, Fz, mass of F^n (fixed
   body) or Fx, Fy, torque about z, mass (turning body) */
int orc3a_step(orc3a *o, const double *F, double *Fo, double *diag) {
  if (o->cfg.motion != 0 && o->cfg.body_kind != 0) return step3a_moving(o, F, Fo, diag);
  int nvel = o->vel.nvel, n = o->nleaf;
  size_t tot = (size_t)n * nvel;
  double *Fm = malloc(tot * sizeof(double));
  memcpy(Fm, F, tot * sizeof(double));
  merge3a(o, Fm);
  if (diag) {
    double Fw[3] = {0, 0, 0}, mass = 0.0;
    for (int k = 0; k < n; ++k)
      if (o->sw[k] > 0.0) wall_force3(&o->vel, Fm + (size_t)o->master[k] * nvel, o->nw3 + 3 * k, o->sw[k], Fw);
    for (int m = 0; m < n; ++m) {
      if (o->master[m] != m) continue;
      double sm = 0.0;
      for (int p = 0; p < nvel; ++p) sm += Fm[(size_t)m * nvel + p] * o->vel.w;
      mass += o->vcv[m] * sm;
    }
    diag[0] = Fw[0]; diag[1] = Fw[1]; diag[2] = Fw[2]; diag[3] = mass;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int m = 0; m < n; ++m) {
    if (o->master[m] != m) continue;
    scheme3a(o, Fm, m, Fo + (size_t)m * nvel);
  }
  for (int c = 0; c < n; ++c) {
    int m = o->master[c];
    if (m < 0) memset(Fo + (size_t)c * nvel, 0, nvel * sizeof(double));
    else if (m != c) memcpy(Fo + (size_t)c * nvel, Fo + (size_t)m * nvel, nvel * sizeof(double));
  }
  free(Fm);
  return 0;
}

/* Mesh adaptation (Section 5.1): the mesh is rebuilt for the body at its
   current angle; the old leaves, with their gas volumes at that angle, are
   kept for orc3a_remap. */
int orc3a_adapt(orc3a *o) {
  free(o->plvl); free(o->pijk); free(o->pvbar); free(o->ptab);
  o->pn = o->nleaf;
  o->plvl = o->lvl; o->pijk = o->ijk; o->ptab = o->tab;
  if (o->vbar1) { o->pvbar = o->vbar1; o->vbar1 = NULL; }
  else { o->pvbar = malloc(o->nleaf * sizeof(double)); memcpy(o->pvbar, o->vbar, o->nleaf * sizeof(double)); }
  o->lvl = NULL; o->ijk = NULL; o->tab = NULL;
  free_mesh3a(o);
  return build3a(o);
}

/* The state carried from the previous mesh to the current one: a leaf that
   is also an old leaf keeps its value; a leaf inside an old leaf takes its
   value (prolongation, 0th order); a leaf covering old leaves takes their
   gas-volume weighted mean, summed in old-leaf order (restriction).  Solid
   leaves are 0. */
void orc3a_remap(const orc3a *o, const double *Fold, double *Fnew) {
  int nvel = o->vel.nvel;
  for (int q = 0; q < o->nleaf; ++q) {
    double *dst = Fnew + (size_t)q * nvel;
    if (o->type[q] == SOLID) { memset(dst, 0, nvel * sizeof(double)); continue; }
    int l = o->lvl[q], i = o->ijk[3 * q], j = o->ijk[3 * q + 1], k = o->ijk[3 * q + 2];
    int src = find_leaf3(o->ptab, o->pn, l, i, j, k);
    for (int a = l - 1; src < 0 && a >= 0; --a)
      src = find_leaf3(o->ptab, o->pn, a, i >> (l - a), j >> (l - a), k >> (l - a));
    if (src >= 0) { memcpy(dst, Fold + (size_t)src * nvel, nvel * sizeof(double)); continue; }
    double W = 0.0;
    memset(dst, 0, nvel * sizeof(double));
    for (int r = 0; r < o->pn; ++r) {
      int sh = o->plvl[r] - l;
      if (sh <= 0) continue;
      if ((o->pijk[3 * r] >> sh) != i || (o->pijk[3 * r + 1] >> sh) != j || (o->pijk[3 * r + 2] >> sh) != k) continue;
      W += o->pvbar[r];
      for (int p = 0; p < nvel; ++p) dst[p] += o->pvbar[r] * Fold[(size_t)r * nvel + p];
    }
    for (int p = 0; p < nvel; ++p) dst[p] = W > 0.0 ? dst[p] / W : 0.0;
  }
}

/* the body's signed distance at angle th (tests) */
double orc3a_levelset(const orc3a *o, double th, double x, double y, double z) {
  return levelset3(&o->cfg, th, x, y, z);
}
