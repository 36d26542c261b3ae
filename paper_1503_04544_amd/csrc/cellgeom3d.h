// Per-cell 3D cut-cell geometry (Section 5.1; the paper leaves the 3D
// geometry to the reader), shared by the uniform-grid geometry kernels and
// the octree builder.  Rules:
//   * a Cartesian face's gas area is the polygon of its gas corners and the
//     linear crossings on its mixed edges; four crossings reject the face;
//   * the wall face closes the cell, |S_w| n_w = -sum_faces |S_k| n_k, n_w
//     pointing into the solid; its centre is the mean of the edge crossings;
//   * the volume follows from the divergence theorem, V = 1/3 sum |S| (m.n).
// Include after `#pragma clang fp contract(off)` so that host and device
// evaluate the formulas in the order written.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>

#include "ccdvm_impl.h"

namespace ccdvm {

// Signed distance to the body, gas side positive (Appendix A).
//   sphere: radius B.a.
//   vane: the points within r = min(a, b, c) of the box of half-sizes
//     (a, b, c) - r in the body frame, turned by B.theta about the z axis
//     through the centre (a plate with rounded edges); B.ct, B.st hold
//     cos and sin of B.theta.  With q = |p| - (a - r)
//     in the body frame the distance to the box is |max(q, 0)| outside and
//     the largest component of q inside.
__host__ __device__ inline double level_set_3d(const BodyDev& B, double x, double y, double z) {
  const double a = x - B.cx, b = y - B.cy, c = z - B.cz;
  if (B.kind == CC_BODY_SPHERE) return sqrt(a * a + b * b + c * c) - B.a;
  if (B.kind == CC_BODY_VANE) {
    const double ct = B.ct, st = B.st;
    const double p[3] = {ct * a + st * b, -st * a + ct * b, c};
    const double ax[3] = {B.a, B.b, B.c};
    const double r = B.a < (B.b < B.c ? B.b : B.c) ? B.a : (B.b < B.c ? B.b : B.c);
    double out2 = 0.0, qmax = -1e300;
    for (int d = 0; d < 3; ++d) {
      const double q = fabs(p[d]) - (ax[d] - r);
      const double qp = q > 0.0 ? q : 0.0;
      out2 += qp * qp;
      qmax = qmax > q ? qmax : q;
    }
    return sqrt(out2) + (qmax < 0.0 ? qmax : 0.0) - r;
  }
  return 1.0e300;
}

// vertex value with the 1e-10 dx clamp, sign(0) = +1
__host__ __device__ inline double clamp_vertex(double p, double dx) {
  const double floor_ = 1e-10 * dx;
  const double m = fabs(p) > floor_ ? fabs(p) : floor_;
  return p >= 0.0 ? m : -m;
}

// gas polygon of a rectangle [0,h1]x[0,h2] with corner values q (corners in
// the order (0,0), (h1,0), (h1,h2), (0,h2)): area, number of crossed edges
__host__ __device__ inline double face_area(const double q[4], double h1, double h2, int* ncross) {
  const double cs[4] = {0.0, h1, h1, 0.0}, ct[4] = {0.0, 0.0, h2, h2};
  double ps[8], pt[8];
  int np = 0, nc = 0;
  for (int e = 0; e < 4; ++e) {
    const int e1 = (e + 1) & 3;
    const bool ga = q[e] > 0.0, gb = q[e1] > 0.0;
    if (ga) { ps[np] = cs[e]; pt[np] = ct[e]; ++np; }
    if (ga != gb) {
      const double t = q[e] / (q[e] - q[e1]);
      ps[np] = cs[e] + t * (cs[e1] - cs[e]);
      pt[np] = ct[e] + t * (ct[e1] - ct[e]);
      ++np;
      ++nc;
    }
  }
  double A = 0.0;
  for (int k = 0; k < np; ++k) {
    const int k1 = k + 1 == np ? 0 : k + 1;
    A += ps[k] * pt[k1] - ps[k1] * pt[k];
  }
  *ncross = nc;
  return 0.5 * A;
}

struct CellGeo3 {
  int type;        // CellType
  int flags;       // bit0: centre in gas (mean vertex value > thr); bit1: saddle face
  double S[6];     // gas areas x-, x+, y-, y+, z-, z+
  double aw;       // wall area (0 unless cut)
  double n[3];     // wall normal into the solid
  double r[3];     // wall centre relative to the cell's lower corner
  double vbar;     // gas volume
};

// geometry of one cell of sizes h from its 8 vertex values
// q8[a | b << 1 | c << 2] (a, b, c = 0/1 along x, y, z)
__host__ __device__ inline void cell_geometry_3d(const double q8[8], const double h[3], double thr,
                                                 CellGeo3& g) {
  double mn = 1e300, mx = -1e300, sum = 0.0;
  for (int b = 0; b < 8; ++b) {
    mn = fmin(mn, q8[b]);
    mx = fmax(mx, q8[b]);
    sum += q8[b];
  }
  const int type = mn > 0.0 ? TYPE_GAS : (mx < 0.0 ? TYPE_SOLID : TYPE_CUT);
  int flags = sum / 8.0 > thr ? 1 : 0;
  double Aw[3] = {0.0, 0.0, 0.0}, V = 0.0;
  for (int d = 0; d < 3; ++d) {
    const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
    for (int sd = 0; sd < 2; ++sd) {
      double q[4];
      for (int u = 0; u < 4; ++u) {
        int idx[3];
        idx[d] = sd;
        idx[d1] = (u == 1 || u == 2) ? 1 : 0;
        idx[d2] = u >= 2 ? 1 : 0;
        q[u] = q8[idx[0] | (idx[1] << 1) | (idx[2] << 2)];
      }
      int nc;
      const double area = face_area(q, h[d1], h[d2], &nc);
      if (nc == 4) flags |= 2;
      g.S[2 * d + sd] = type == TYPE_SOLID ? 0.0 : area;
      const double sgn = sd ? 1.0 : -1.0;
      Aw[d] -= sgn * area;
      V += area * (sd ? h[d] : 0.0) / 3.0;
    }
  }
  // mean of the crossings on the 12 edges
  double rs[3] = {0.0, 0.0, 0.0};
  int ncx = 0;
  for (int d = 0; d < 3; ++d) {
    const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
    for (int u = 0; u < 4; ++u) {
      int i0[3], i1[3];
      i0[d] = 0; i1[d] = 1;
      i0[d1] = i1[d1] = u & 1;
      i0[d2] = i1[d2] = (u >> 1) & 1;
      const double qa = q8[i0[0] | (i0[1] << 1) | (i0[2] << 2)];
      const double qb = q8[i1[0] | (i1[1] << 1) | (i1[2] << 2)];
      if ((qa > 0.0) != (qb > 0.0)) {
        const double tt = qa / (qa - qb);
        double p3[3];
        p3[d] = tt * h[d];
        p3[d1] = i0[d1] * h[d1];
        p3[d2] = i0[d2] * h[d2];
        rs[0] += p3[0]; rs[1] += p3[1]; rs[2] += p3[2];
        ++ncx;
      }
    }
  }
  const double Sw = sqrt(Aw[0] * Aw[0] + Aw[1] * Aw[1] + Aw[2] * Aw[2]);
  g.aw = 0.0;
  for (int d = 0; d < 3; ++d) { g.n[d] = 0.0; g.r[d] = 0.0; }
  if (type == TYPE_CUT && ncx > 0 && Sw > 0.0) {
    const double r[3] = {rs[0] / ncx, rs[1] / ncx, rs[2] / ncx};
    g.aw = Sw;
    g.n[0] = Aw[0] / Sw; g.n[1] = Aw[1] / Sw; g.n[2] = Aw[2] / Sw;
    V += (r[0] * Aw[0] + r[1] * Aw[1] + r[2] * Aw[2]) / 3.0;
    g.r[0] = r[0]; g.r[1] = r[1]; g.r[2] = r[2];
  }
  g.type = type;
  g.flags = flags;
  g.vbar = type == TYPE_SOLID ? 0.0 : (type == TYPE_GAS ? h[0] * h[1] * h[2] : V);
}

}  // namespace ccdvm
