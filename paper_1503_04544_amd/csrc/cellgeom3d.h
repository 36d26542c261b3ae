// Per-cell 3D cut-cell geometry (Section 5; Appendix A leaves
// its extension to 3D to the reader), used by the uniform-grid geometry kernels and the
// octree builder.  Rules (the 2D virtual-cell rules of Appendix A carried to
// the six faces of a hexahedral cell):
//   * a Cartesian face's gas part is bounded by its gas corners and the linear
//     crossings of the level set on its mixed edges; a face crossed on all
//     four edges rejects the geometry;
//   * the wall face is the surface spanned by the loop of edge crossings; its
//     vector area (n_w pointing into the solid) closes the cell, so it equals
//     minus the sum of the Cartesian faces' outward vector areas;
//   * the wall centre is the mean of the edge crossings;
//   * the gas volume follows from the divergence theorem.
//
// How it is evaluated here:
//   * face areas by the number and position of the gas corners: a corner
//     triangle, a trapezoid on the gas edge, or the face minus the solid
//     corner triangles;
//   * the wall vector area from the crossing loop itself (Newell's formula
//     for a closed polygon, 1/2 sum p_k x p_{k+1}), one chord per crossed
//     face, with the points taken about the wall centre;
//   * the volume as a sum of pyramids with their apex at the wall centre
//     (the wall fan contributes nothing), so each Cartesian face adds
//     1/3 |S| times its distance to the apex.
// Corner k of a cell sits at ((k >> 2) & 1, (k >> 1) & 1, k & 1) in units of
// the cell sizes (x is the high bit).
// Include after `#pragma clang fp contract(off)` so that host and device
// evaluate the formulas in the order written.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>

#include "ccdvm_impl.h"

namespace ccdvm {

// Signed distance to the body, gas side positive (Appendix A).
//   sphere: radius B.a about the centre.
//   vane: the points within r = min(a, b, c) of the box of half-sizes
//     e = (a, b, c) - r, the box turned by B.theta about the z axis through
//     the centre (B.ct, B.st hold cos and sin of B.theta).  The nearest point
//     of the box to a point p outside it is p clamped to [-e, e]; inside, the
//     distance is the smallest slack e_d - |p_d|.
__host__ __device__ inline double level_set_3d(const BodyDev& B, double x, double y, double z) {
  const double dx = x - B.cx, dy = y - B.cy, dz = z - B.cz;
  if (B.kind == CC_BODY_SPHERE) return sqrt(dx * dx + dy * dy + dz * dz) - B.a;
  if (B.kind == CC_BODY_VANE) {
    const double rr = fmin(B.a, fmin(B.b, B.c));
    const double pb[3] = {B.ct * dx + B.st * dy, B.ct * dy - B.st * dx, dz};
    const double e[3] = {B.a - rr, B.b - rr, B.c - rr};
    bool inside = true;
    double gap2 = 0.0, slack = 1e300;
    for (int d = 0; d < 3; ++d) {
      const double ad = fabs(pb[d]);
      if (ad > e[d]) {
        inside = false;
        const double o = ad - e[d];
        gap2 += o * o;
      } else {
        slack = fmin(slack, e[d] - ad);
      }
    }
    return (inside ? -slack : sqrt(gap2)) - rr;
  }
  return 1.0e300;
}

// vertex value with the 1e-10 dx floor on its magnitude, sign(0) = +1
__host__ __device__ inline double clamp_vertex(double p, double dx) {
  const double m = fmax(fabs(p), 1e-10 * dx);
  return p < 0.0 ? -m : m;
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

namespace cg3 {

// The six faces in the order x-, x+, y-, y+, z-, z+: axis, and the four
// corners counter-clockwise about the outward normal.
struct FaceDef { int axis; int hi; int c[4]; };
__host__ __device__ inline FaceDef face_def(int f) {
  switch (f) {
    case 0: return {0, 0, {0, 1, 3, 2}};
    case 1: return {0, 1, {4, 6, 7, 5}};
    case 2: return {1, 0, {0, 4, 5, 1}};
    case 3: return {1, 1, {2, 3, 7, 6}};
    case 4: return {2, 0, {0, 2, 6, 4}};
    default: return {2, 1, {1, 5, 7, 3}};
  }
}

// axis along which corners a and b (neighbours) differ
__host__ __device__ inline int edge_axis(int a, int b) {
  const int x = a ^ b;
  return x == 4 ? 0 : (x == 2 ? 1 : 2);
}

// edge slot of the edge between neighbouring corners a and b: its axis and
// the lower corner's remaining two bits
__host__ __device__ inline int edge_slot(int a, int b) {
  const int ax = edge_axis(a, b);
  const int lo = a < b ? a : b;
  int rest;
  if (ax == 0) rest = lo & 3;
  else if (ax == 1) rest = ((lo >> 2) << 1) | (lo & 1);
  else rest = lo >> 1;
  return 4 * ax + rest;
}

// distance from corner a to the crossing on its edge towards b (signs of
// qa and qb differ), for an edge of length L
__host__ __device__ inline double to_cross(double qa, double qb, double L) {
  return L * (qa / (qa - qb));
}

}  // namespace cg3

// geometry of one cell of sizes h from its 8 vertex values q[k], corner k as
// in the header comment
__host__ __device__ inline void cell_geometry_3d(const double q[8], const double h[3], double thr,
                                                 CellGeo3& g) {
  using namespace cg3;
  bool any_gas = false, any_solid = false;
  double qsum = 0.0;
  for (int k = 0; k < 8; ++k) {
    any_gas |= q[k] > 0.0;
    any_solid |= !(q[k] > 0.0);
    qsum += q[k];
  }
  g.type = !any_solid ? TYPE_GAS : (!any_gas ? TYPE_SOLID : TYPE_CUT);
  g.flags = qsum * 0.125 > thr ? 1 : 0;
  g.aw = 0.0;
  for (int d = 0; d < 3; ++d) { g.n[d] = 0.0; g.r[d] = 0.0; }
  if (g.type == TYPE_SOLID) {
    for (int f = 0; f < 6; ++f) g.S[f] = 0.0;
    g.vbar = 0.0;
    return;
  }
  if (g.type == TYPE_GAS) {
    g.S[0] = g.S[1] = h[1] * h[2];
    g.S[2] = g.S[3] = h[0] * h[2];
    g.S[4] = g.S[5] = h[0] * h[1];
    g.vbar = h[0] * h[1] * h[2];
    return;
  }

  // crossing point of every mixed edge, from the edge's lower corner
  double X[12][3];
  double m[3] = {0.0, 0.0, 0.0};
  int ncross = 0;
  for (int a = 0; a < 8; ++a)
    for (int ax = 0; ax < 3; ++ax) {
      const int bit = 4 >> ax;
      if (a & bit) continue;
      const int b = a | bit;
      if ((q[a] > 0.0) == (q[b] > 0.0)) continue;
      const int s = edge_slot(a, b);
      const double p0[3] = {(a & 4) ? h[0] : 0.0, (a & 2) ? h[1] : 0.0, (a & 1) ? h[2] : 0.0};
      for (int d = 0; d < 3; ++d) X[s][d] = p0[d];
      X[s][ax] = to_cross(q[a], q[b], h[ax]);
      for (int d = 0; d < 3; ++d) m[d] += X[s][d];
      ++ncross;
    }
  for (int d = 0; d < 3; ++d) m[d] /= (double)ncross;

  double W[3] = {0.0, 0.0, 0.0};   // wall vector area
  double vol3 = 0.0;               // three times the volume
  for (int f = 0; f < 6; ++f) {
    const FaceDef F = face_def(f);
    const int u1 = F.axis == 0 ? 1 : 0, u2 = F.axis == 2 ? 1 : 2;
    const double L1 = h[u1], L2 = h[u2];
    bool gas[4];
    int ngas = 0;
    for (int k = 0; k < 4; ++k) { gas[k] = q[F.c[k]] > 0.0; ngas += gas[k]; }
    // length of the edge from corner slot k to k + 1
    auto elen = [&](int k) { return h[edge_axis(F.c[k], F.c[(k + 1) & 3])]; };
    // distance from corner slot k to the crossing towards slot k + dk
    auto dist = [&](int k, int dk) {
      const int k2 = (k + dk) & 3;
      const int e = dk == 1 ? k : k2;
      return to_cross(q[F.c[k]], q[F.c[k2]], elen(e));
    };
    double A;
    if (ngas == 4) {
      A = L1 * L2;
    } else if (ngas == 0) {
      A = 0.0;
    } else if (ngas == 1 || ngas == 3) {
      int k = 0;
      while (gas[k] != (ngas == 1)) ++k;
      const double tri = 0.5 * dist(k, 1) * dist(k, 3);
      A = ngas == 1 ? tri : L1 * L2 - tri;
    } else {
      int k = 0;
      while (k < 4 && !(gas[k] && gas[(k + 1) & 3])) ++k;
      if (k < 4) {                       // gas edge from slot k to k + 1: trapezoid
        A = elen(k) * 0.5 * (dist(k, 3) + dist((k + 1) & 3, 1));
      } else {                           // opposite gas corners: both edges crossed twice
        g.flags |= 2;
        const int s0 = gas[0] ? 1 : 0, s1 = s0 + 2;
        A = L1 * L2 - 0.5 * dist(s0, 1) * dist(s0, 3) - 0.5 * dist(s1, 1) * dist(s1, 3);
      }
    }
    g.S[f] = A;
    // pyramid from the wall centre over this face: distance along the
    // outward normal from the apex to the face plane
    const double hgt = F.hi ? h[F.axis] - m[F.axis] : m[F.axis];
    vol3 += A * hgt;

    // chords of the wall loop on this face: walking the corners in order
    // from a gas corner, the gas part leaves at X_out and comes back at X_in;
    // the wall runs the chord the other way, adding 1/2 X_in x X_out
    if (ngas == 0 || ngas == 4) continue;
    int k0 = 0;
    while (!gas[k0]) ++k0;
    double xo[3] = {0.0, 0.0, 0.0};
    for (int t = 0; t < 4; ++t) {
      const int ka = (k0 + t) & 3, kb = (ka + 1) & 3;
      if (gas[ka] == gas[kb]) continue;
      const double* P = X[edge_slot(F.c[ka], F.c[kb])];
      const double p[3] = {P[0] - m[0], P[1] - m[1], P[2] - m[2]};
      if (gas[ka]) {
        xo[0] = p[0]; xo[1] = p[1]; xo[2] = p[2];
      } else {
        W[0] += 0.5 * (p[1] * xo[2] - p[2] * xo[1]);
        W[1] += 0.5 * (p[2] * xo[0] - p[0] * xo[2]);
        W[2] += 0.5 * (p[0] * xo[1] - p[1] * xo[0]);
      }
    }
  }
  g.vbar = vol3 / 3.0;
  const double area = sqrt(W[0] * W[0] + W[1] * W[1] + W[2] * W[2]);
  if (area > 0.0) {
    g.aw = area;
    for (int d = 0; d < 3; ++d) { g.n[d] = W[d] / area; g.r[d] = m[d]; }
  }
}

}  // namespace ccdvm
