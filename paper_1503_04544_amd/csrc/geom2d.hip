// Device construction of the 2D cut-cell geometry (Appendix A of the paper):
// vertex level set with the 1e-10 dx clamp (A.1), cell types from the sign
// pattern (A.1), gas lengths of the Cartesian edges by linear interpolation of
// the crossing points (A.2), wall edge by closure of the virtual cell with the
// normal pointing into the solid (A.2), virtual-cell area (A.4), master search
// with test (ii) and algorithm (fusion) (A.3), control-volume areas (A.4) and
// the compact list of control volumes handled by the cut-cell kernel.
//
// Everything is a pure function of the level set, so building it on the GPU
// costs a handful of small launches; a moving body rebuilds it every step.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include "ccdvm_impl.h"

namespace ccdvm {
namespace {

// Signed distance to the ellipse X^2/a^2 + Y^2/b^2 = 1 (negative inside).
// The nearest point is (a^2 X/(a^2+t), b^2 Y/(b^2+t)), t the unique root of
// G(t) = (aX/(a^2+t))^2 + (bY/(b^2+t))^2 - 1 on t > -min(a, b)^2, G
// decreasing and convex there: Newton from the right of the root converges
// monotonically; a bracket guards against round-off.
__device__ double ellipse_signed_distance(double a, double b, double x, double y) {
  double X = fabs(x), Y = fabs(y);
  if (b > a) { double t = a; a = b; b = t; t = X; X = Y; Y = t; }
  const double a2 = a * a, b2 = b * b;
  const double q = X * X / a2 + Y * Y / b2 - 1.0;
  double px, py;
  if (Y == 0.0) {
    // on the major axis: interior points may have their nearest point off-axis
    double lim = (a2 - b2) / a;
    if (X < lim) {
      double xs = a2 * X / (a2 - b2);
      px = xs;
      double r = 1.0 - (xs / a) * (xs / a);
      py = b * sqrt(r > 0.0 ? r : 0.0);
    } else {
      px = a; py = 0.0;
    }
  } else if (X == 0.0) {
    px = 0.0; py = b;
  } else {
    double lo = -b2;                               // G(lo+) = +inf
    double t = fmax(a * X, b * Y) - b2;            // G(t) <= 0 here
    if (t < lo) t = lo;
    double hi = t + a * X + b * Y + 1.0;           // G(hi) < 0 surely
    // start from the right end of the bracket
    t = hi;
    for (int it = 0; it < 200; ++it) {
      double ra = a * X / (a2 + t), rb = b * Y / (b2 + t);
      double G = ra * ra + rb * rb - 1.0;
      if (G > 0.0) lo = t; else hi = t;
      double dG = -2.0 * (ra * ra / (a2 + t) + rb * rb / (b2 + t));
      double tn = t - G / dG;
      if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
      if (tn == t || hi - lo <= 1e-17 * fabs(hi)) { t = tn; break; }
      t = tn;
    }
    px = a2 * X / (a2 + t);
    py = b2 * Y / (b2 + t);
  }
  double d = hypot(px - X, py - Y);
  return q < 0.0 ? -d : d;
}

__device__ double level_set_2d(const BodyDev& B, double x, double y, double cx,
                               double cy, double th) {
  double ex = x - cx, ey = y - cy;
  switch (B.kind) {
    case CC_BODY_CIRCLE: return hypot(ex, ey) - B.a;
    case CC_BODY_CAVITY: return B.a - hypot(ex, ey);
    case CC_BODY_HALFPLANE: return ex * cos(th) + ey * sin(th);
    case CC_BODY_ELLIPSE: {
      double c = cos(th), s = sin(th);
      return ellipse_signed_distance(B.a, B.b, c * ex + s * ey, -s * ex + c * ey);
    }
    default: return 1.0e300;
  }
}

// vertices [i0, i0+ni] x [j0, j0+nj] of a box of cells; pose = (cx, cy, theta)
__global__ void k_phi2d(Geo2D G, BodyDev B, const double* __restrict__ pose, Box2D bx) {
  int nvx = G.nx + 1;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (bx.ni + 1) * (bx.nj + 1)) return;
  int a = bx.i0 + t % (bx.ni + 1), b = bx.j0 + t / (bx.ni + 1);
  double p = level_set_2d(B, G.x0 + a * G.dx, G.y0 + b * G.dy, pose[0], pose[1], pose[2]);
  t = b * nvx + a;
  double floor_ = 1e-10 * G.dx;
  double m = fabs(p) > floor_ ? fabs(p) : floor_;
  G.phi[t] = p >= 0.0 ? m : -m;
}

// gas length of an edge of length h whose ends carry level-set values pa
// (s = 0) and pb (s = h); *s receives the crossing abscissa on a mixed edge
__device__ inline double gas_len(double pa, double pb, double h, bool* mixed, double* s) {
  bool ga = pa > 0.0, gb = pb > 0.0;
  *mixed = ga != gb;
  if (ga && gb) return h;
  if (!ga && !gb) return 0.0;
  double sc = h * pa / (pa - pb);
  *s = sc;
  return ga ? sc : h - sc;
}

__global__ void k_cell2d(Geo2D G, Box2D bx) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= bx.ni * bx.nj) return;
  int i = bx.i0 + t % bx.ni, j = bx.j0 + t / bx.ni;
  int c = j * G.nx + i;
  int nvx = G.nx + 1;
  double p00 = G.phi[j * nvx + i], p10 = G.phi[j * nvx + i + 1];
  double p11 = G.phi[(j + 1) * nvx + i + 1], p01 = G.phi[(j + 1) * nvx + i];
  double mn = fmin(fmin(p00, p10), fmin(p11, p01));
  double mx = fmax(fmax(p00, p10), fmax(p11, p01));
  int type = mn > 0.0 ? TYPE_GAS : (mx < 0.0 ? TYPE_SOLID : TYPE_CUT);
  const double dx = G.dx, dy = G.dy;
  bool mr, ml, mt, mb;
  double sr = 0, sl = 0, st = 0, sb = 0;
  double Lr = gas_len(p10, p11, dy, &mr, &sr);   // right edge, bottom -> top
  double Ll = gas_len(p00, p01, dy, &ml, &sl);   // left edge
  double Lt = gas_len(p01, p11, dx, &mt, &st);   // top edge, left -> right
  double Lb = gas_len(p00, p10, dx, &mb, &sb);   // bottom edge
  int nmix = (int)mr + (int)ml + (int)mt + (int)mb;
  int flags = 0;
  if (0.25 * (p00 + p10 + p11 + p01) > 1e-12 * dx) flags |= 1;
  if (nmix == 4) flags |= 2;
  // polygon of the virtual cell, counter-clockwise from the lower-left
  // corner, in coordinates relative to that corner
  double vx[8], vy[8];
  int nvtx = 0;
  if (p00 > 0.0) { vx[nvtx] = 0.0; vy[nvtx] = 0.0; ++nvtx; }
  if (mb) { vx[nvtx] = sb; vy[nvtx] = 0.0; ++nvtx; }
  if (p10 > 0.0) { vx[nvtx] = dx; vy[nvtx] = 0.0; ++nvtx; }
  if (mr) { vx[nvtx] = dx; vy[nvtx] = sr; ++nvtx; }
  if (p11 > 0.0) { vx[nvtx] = dx; vy[nvtx] = dy; ++nvtx; }
  if (mt) { vx[nvtx] = st; vy[nvtx] = dy; ++nvtx; }
  if (p01 > 0.0) { vx[nvtx] = 0.0; vy[nvtx] = dy; ++nvtx; }
  if (ml) { vx[nvtx] = 0.0; vy[nvtx] = sl; ++nvtx; }
  double area = 0.0;
  for (int k = 0; k < nvtx; ++k) {
    int k1 = k + 1 == nvtx ? 0 : k + 1;
    area += vx[k] * vy[k1] - vx[k1] * vy[k];
  }
  area *= 0.5;
  // wall edge: |L_w| n_w closes the polygon of Cartesian edges
  double ddx = Lr - Ll, ddy = Lt - Lb;
  double lw = 0.0, nx_ = 0.0, ny_ = 0.0, rx = 0.0, ry = 0.0;
  if (type == TYPE_CUT && nmix == 2) {
    lw = sqrt(ddx * ddx + ddy * ddy);
    if (lw > 0.0) {
      nx_ = -ddx / lw; ny_ = -ddy / lw;
      double cxs = 0.0, cys = 0.0;
      if (mr) { cxs += dx; cys += sr; }
      if (ml) { cxs += 0.0; cys += sl; }
      if (mt) { cxs += st; cys += dy; }
      if (mb) { cxs += sb; cys += 0.0; }
      rx = 0.5 * cxs; ry = 0.5 * cys;
    }
  }
  G.type[c] = type;
  G.flags[c] = flags;
  G.lxp[c] = Lr; G.lxm[c] = Ll; G.lyp[c] = Lt; G.lym[c] = Lb;
  G.lw[c] = lw; G.nwx[c] = nx_; G.nwy[c] = ny_;
  G.rwx[c] = G.x0 + i * dx + rx;
  G.rwy[c] = G.y0 + j * dy + ry;
  G.sbar[c] = type == TYPE_SOLID ? 0.0 : (type == TYPE_GAS ? dx * dy : area);
}

__global__ void k_master2d(Geo2D G, Box2D bx) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= bx.ni * bx.nj) return;
  int i = bx.i0 + t % bx.ni, j = bx.j0 + t / bx.ni;
  int c = j * G.nx + i;
  if (G.type[c] == TYPE_SOLID) { G.master[c] = -1; return; }
  int seen[kHopCap + 1];
  seen[0] = c;
  int hops = 0;
  bool bad = false;
  while (!(G.flags[j * G.nx + i] & 1)) {
    if (hops == kHopCap || !hop2d(G, i, j)) { bad = true; break; }
    ++hops;
    int nc = j * G.nx + i;
    for (int h = 0; h < hops; ++h) bad |= seen[h] == nc;
    if (bad) break;
    seen[hops] = nc;
  }
  G.master[c] = j * G.nx + i;
  if (bad) atomicOr(&G.counts[3], 1);
  if (G.flags[c] & 2) atomicOr(&G.counts[3], 2);
}

// control-volume area and kind; members of a control volume are cut cells
// within kHopCap cells of their master, and a master owning members touches
// a cut cell
__global__ void k_cv2d(Geo2D G, Box2D bx) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= bx.ni * bx.nj) return;
  int c = (bx.j0 + t / bx.ni) * G.nx + bx.i0 + t % bx.ni;
  int m = G.master[c];
  if (m < 0) { G.kind[c] = KIND_SOLID; G.scv[c] = 0.0; return; }
  if (m != c) { G.kind[c] = KIND_MEMBER; G.scv[c] = 0.0; return; }
  int i = c % G.nx, j = c / G.nx;
  bool near_cut = false;
  for (int dj = -1; dj <= 1; ++dj)
    for (int di = -1; di <= 1; ++di) {
      int ii = i + di, jj = j + dj;
      if (ii >= 0 && jj >= 0 && ii < G.nx && jj < G.ny) near_cut |= G.type[jj * G.nx + ii] == TYPE_CUT;
    }
  double S = 0.0;
  int cnt = 0;
  if (!near_cut) {
    S = G.sbar[c]; cnt = 1;
  } else {
    for (int jj = max(j - kHopCap, 0); jj <= min(j + kHopCap, G.ny - 1); ++jj)
      for (int ii = max(i - kHopCap, 0); ii <= min(i + kHopCap, G.nx - 1); ++ii) {
        int k = jj * G.nx + ii;
        if (G.master[k] == c) { S += G.sbar[k]; ++cnt; }
      }
  }
  G.scv[c] = S;
  G.kind[c] = (G.type[c] == TYPE_GAS && cnt == 1) ? KIND_REGULAR : KIND_IRREGULAR;
  if (cnt > kMaxMembers) atomicOr(&G.counts[3], 4);
}

// Single-block deterministic compaction: list of irregular masters in
// ascending cell order, CSR of their members (ascending), population counts.
// The box cells are taken kScanPer consecutive ones per thread and round,
// the list by a block scan per round.  Members are counted and placed through integer
// atomics on the per-cell scratch, and every member list is then sorted, so
// the result does not depend on the order of the atomics.
__global__ void __launch_bounds__(1024) k_compact2d(Geo2D G, Box2D bx) {
  __shared__ int sh[1024];
  const int t = threadIdx.x, nth = blockDim.x;
  const int nbox = bx.ni * bx.nj;
  // box index -> cell index, ascending in the cell order
  auto cell = [&](int u) { return (bx.j0 + u / bx.ni) * G.nx + bx.i0 + u % bx.ni; };
  // a listed master: irregular and inside the box
  auto listed = [&](int m) {
    if (m < 0) return false;
    const int i = m % G.nx - bx.i0, j = m / G.nx - bx.j0;
    return i >= 0 && i < bx.ni && j >= 0 && j < bx.nj && G.kind[m] == KIND_IRREGULAR;
  };
  int carry = 0, nmem = 0, nsol = 0;
  for (int base = 0; base < nbox; base += nth * kScanPer) {
    int c[kScanPer], k[kScanPer], cnt = 0;
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
      const int u = base + t * kScanPer + e;
      c[e] = 0;
      k[e] = -1;
      if (u < nbox) { c[e] = cell(u); k[e] = G.kind[c[e]]; }
      nmem += k[e] == KIND_MEMBER;
      nsol += k[e] == KIND_SOLID;
      cnt += k[e] == KIND_IRREGULAR;
    }
    int tot;
    int w = carry + block_scan_excl(cnt, sh, &tot);
#pragma unroll
    for (int e = 0; e < kScanPer; ++e)
      if (k[e] == KIND_IRREGULAR) { G.irr[w++] = c[e]; G.aux[c[e]] = 0; }
    carry += tot;
  }
  const int tot_irr = carry;
  int tot_mem, tot_sol;
  block_scan_excl(nmem, sh, &tot_mem);
  block_scan_excl(nsol, sh, &tot_sol);
  if (t == 0) { G.counts[0] = tot_irr; G.counts[1] = tot_mem; G.counts[2] = tot_sol; }
  // member counts of the listed masters
  for (int u = t; u < nbox; u += nth) {
    const int m = G.master[cell(u)];
    if (listed(m)) atomicAdd(&G.aux[m], 1);
  }
  __syncthreads();
  // CSR pointers by a chunked scan; each count becomes its list's cursor
  carry = 0;
  for (int base = 0; base < tot_irr; base += nth) {
    const int q = base + t;
    int cnt = 0, m = 0;
    if (q < tot_irr) { m = G.irr[q]; cnt = load_l2(&G.aux[m]); }
    int tot;
    const int ex = block_scan_excl(cnt, sh, &tot);
    if (q < tot_irr) { G.mptr[q] = carry + ex; G.aux[m] = carry + ex; }
    carry += tot;
  }
  if (t == 0) G.mptr[tot_irr] = carry;
  __syncthreads();
  for (int u = t; u < nbox; u += nth) {
    const int c = cell(u), m = G.master[c];
    if (listed(m)) G.mem[atomicAdd(&G.aux[m], 1)] = c;
  }
  __syncthreads();
  for (int q = t; q < tot_irr; q += nth) sort_cells(G.mem + G.mptr[q], G.mptr[q + 1] - G.mptr[q]);
}

// velocity nodes (midpoints of the velocity box) and farfield table
__global__ void k_tables2d(Geo2D G, double vmin, double dv, double rho, double ux,
                           double uy, double T) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < G.N) G.vnode[p] = vmin + (p + 0.5) * dv;
  if (p >= G.nvel) return;
  double vx = vmin + (p % G.N + 0.5) * dv, vy = vmin + (p / G.N + 0.5) * dv;
  double ex = vx - ux, ey = vy - uy;
  double f = rho / (2.0 * M_PI * T) * exp(-(ex * ex + ey * ey) / (2.0 * T));
  G.ghost[p] = make_double2(f, 0.5 * T * f);
}

// Outflow rate phi of eq. (phiCFL) of each cut or merged control volume
// divided by its area, maximised over the velocity grid.  phi is a sum of
// terms of the form |L| max(a . v + b, 0), convex in v, so its largest value
// on the grid is taken at one of the four corner nodes (vlo|vhi, vlo|vhi).
// The wall velocity is the rigid motion u_w = (ux, uy) + om (r - c)^perp of
// eq. (uwDD).  The maximum over the control volumes is folded into *out as
// the bit pattern of a non-negative double (order-preserving).
__global__ void k_cfl2d(Geo2D G, int nirr, double vlo, double vhi, double ux, double uy, double om,
                        double cx, double cy, unsigned long long* out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nirr) return;
  const int m = G.irr[q];
  double best = 0.0;
  for (int corner = 0; corner < 4; ++corner) {
    const double v1 = (corner & 1) ? vhi : vlo, v2 = (corner & 2) ? vhi : vlo;
    double phi = 0.0;
    for (int e = G.mptr[q]; e < G.mptr[q + 1]; ++e) {
      const int k = G.mem[e];
      phi += G.lxp[k] * fmax(v1, 0.0) - G.lxm[k] * fmin(v1, 0.0) + G.lyp[k] * fmax(v2, 0.0) -
             G.lym[k] * fmin(v2, 0.0);
      if (G.lw[k] > 0.0) {
        const double uwx = ux - om * (G.rwy[k] - cy), uwy = uy + om * (G.rwx[k] - cx);
        phi += G.lw[k] * fmax((v1 - uwx) * G.nwx[k] + (v2 - uwy) * G.nwy[k], 0.0);
      }
    }
    best = fmax(best, phi / G.scv[m]);
  }
  atomicMax(out, (unsigned long long)__double_as_longlong(best));
}

}  // namespace

// Largest outflow rate per unit area of eq. (eq-CFL) over the cut and merged
// control volumes of the current geometry (velocity extremes vlo, vhi; body
// state s = cx, cy, theta, ux, uy, omega); synchronises the stream.  `word`
// is a device word of scratch memory.
hipError_t cfl_rate_2d(cc_ctx* ctx, double vlo, double vhi, const double* s, double* rate) {
  const Geo2D& G = ctx->g2;
  unsigned long long* word = reinterpret_cast<unsigned long long*>(ctx->s.red);
  hipError_t e = hipMemsetAsync(word, 0, sizeof(unsigned long long), ctx->stream);
  if (e != hipSuccess) return e;
  if (ctx->n_irr > 0)
    k_cfl2d<<<(ctx->n_irr + 127) / 128, 128, 0, ctx->stream>>>(G, ctx->n_irr, vlo, vhi, s[3], s[4], s[5], s[0],
                                                               s[1], word);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  unsigned long long bits = 0;
  e = hipMemcpyAsync(&bits, word, sizeof(bits), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  double r;
  memcpy(&r, &bits, sizeof(r));
  *rate = r;
  return e;
}

BodyDev body_dev(const cc_ctx* ctx) {
  BodyDev B{};
  B.kind = ctx->body.kind;
  B.a = ctx->body.axes[0]; B.b = ctx->body.axes[1];
  B.t_wall = ctx->body.t_wall;
  return B;
}

// Geometry of G for the pose stored at `pose` (device), inside box bx (the
// cells outside it are gas cells of unchanged geometry).
hipError_t build_geometry_box_2d(cc_ctx* ctx, Geo2D& G, const double* pose, Box2D bx) {
  BodyDev B = body_dev(ctx);
  hipStream_t s = ctx->stream;
  hipError_t e = hipMemsetAsync(G.counts, 0, 3 * sizeof(int), s);
  if (e != hipSuccess) return e;
  int nv = (bx.ni + 1) * (bx.nj + 1), nc = bx.ni * bx.nj;
  k_phi2d<<<(nv + 255) / 256, 256, 0, s>>>(G, B, pose, bx);
  k_cell2d<<<(nc + 255) / 256, 256, 0, s>>>(G, bx);
  k_master2d<<<(nc + 255) / 256, 256, 0, s>>>(G, bx);
  k_cv2d<<<(nc + 255) / 256, 256, 0, s>>>(G, bx);
  k_compact2d<<<1, 1024, 0, s>>>(G, bx);
  return hipGetLastError();
}

hipError_t build_geometry_2d(cc_ctx* ctx, Geo2D& G, const double* pose) {
  hipError_t e = hipMemsetAsync(G.counts, 0, 4 * sizeof(int), ctx->stream);
  if (e != hipSuccess) return e;
  Box2D all{0, 0, G.nx, G.ny};
  e = build_geometry_box_2d(ctx, G, pose, all);
  if (e != hipSuccess) return e;
  const double* in = ctx->cfg.inflow;
  int nt = G.nvel > G.N ? G.nvel : G.N;
  k_tables2d<<<(nt + 255) / 256, 256, 0, ctx->stream>>>(G, ctx->cfg.vmin, ctx->dv, in[0], in[1],
                                                       in[2], in[4]);
  return hipGetLastError();
}

}  // namespace ccdvm
