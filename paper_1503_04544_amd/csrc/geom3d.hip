// Device construction of the 3D cut-cell geometry (Section 5.1, fixed body).
// The paper leaves the 3D geometry to the reader; the rules used here:
//   * vertex level set with the 1e-10 dx clamp, sign(0) = +1;
//   * a Cartesian face's gas area is the polygon of its gas corners and the
//     linear crossings on its mixed edges (the 2D virtual-cell rule on the
//     face's four vertices); a face crossed on all four edges rejects the
//     geometry;
//   * the wall face closes the cell, |S_w| n_w = -sum_faces |S_k| n_k, with
//     n_w pointing into the solid; its centre is the mean of the edge
//     crossings;
//   * the volume follows from the divergence theorem, V = 1/3 sum |S| (m.n);
//   * master search: centre in gas when the mean of the 8 vertex values
//     exceeds 1e-12 dx, otherwise hop across the largest face shared with a
//     cell of the domain (ties within 1e-12 broken in the order x+, x-, y+,
//     y-, z+, z-), at most 4 hops, no revisits.
// Floating-point contraction is off in this file so that the tables are the
// correctly rounded evaluation of these formulas in the order written, which
// keeps tie decisions reproducible.
#include <hip/hip_runtime.h>

#include <math.h>

#include "ccdvm_impl.h"

#pragma clang fp contract(off)

namespace ccdvm {
namespace {

__device__ inline double level_set_3d(const BodyDev& B, double x, double y, double z) {
  if (B.kind == CC_BODY_SPHERE) {
    const double a = x - B.cx, b = y - B.cy, c = z - B.cz;
    return sqrt(a * a + b * b + c * c) - B.a;
  }
  return 1.0e300;
}

__global__ void k_phi3d(Geo3D G, BodyDev B) {
  const long long nvx = G.nx + 1, nvy = G.ny + 1, nvz = G.nz + 1;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nvx * nvy * nvz) return;
  const int a = (int)(t % nvx), b = (int)((t / nvx) % nvy), c = (int)(t / (nvx * nvy));
  const double p = level_set_3d(B, G.x0 + a * G.dx, G.y0 + b * G.dy, G.z0 + c * G.dz);
  const double floor_ = 1e-10 * G.dx;
  const double m = fabs(p) > floor_ ? fabs(p) : floor_;
  G.phi[t] = p >= 0.0 ? m : -m;
}

// vertex value of corner (bx, by, bz) of the cell at (i, j, k)
__device__ inline double vtx(const Geo3D& G, int i, int j, int k, int bx, int by, int bz) {
  const long long nvx = G.nx + 1, nvy = G.ny + 1;
  return G.phi[((long long)(k + bz) * nvy + (j + by)) * nvx + (i + bx)];
}

// gas polygon of a rectangle [0,h1]x[0,h2] with corner values q (corners in
// the order (0,0), (h1,0), (h1,h2), (0,h2)): area, number of crossed edges
__device__ inline double face_area(const double q[4], double h1, double h2, int* ncross) {
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

__global__ void k_cell3d(Geo3D G) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= G.ncell) return;
  const int i = t % G.nx, j = (t / G.nx) % G.ny, k = t / (G.nx * G.ny);
  double q8[8];
  double mn = 1e300, mx = -1e300, sum = 0.0;
  for (int b = 0; b < 8; ++b) {
    q8[b] = vtx(G, i, j, k, b & 1, (b >> 1) & 1, (b >> 2) & 1);
    mn = fmin(mn, q8[b]);
    mx = fmax(mx, q8[b]);
    sum += q8[b];
  }
  const int type = mn > 0.0 ? TYPE_GAS : (mx < 0.0 ? TYPE_SOLID : TYPE_CUT);
  const double h[3] = {G.dx, G.dy, G.dz};
  int flags = sum / 8.0 > 1e-12 * G.dx ? 1 : 0;
  double S[6], Aw[3] = {0.0, 0.0, 0.0}, V = 0.0;
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
      S[2 * d + sd] = type == TYPE_SOLID ? 0.0 : area;
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
  double aw = 0.0, n0 = 0.0, n1 = 0.0, n2 = 0.0, r0 = 0.0, r1 = 0.0, r2 = 0.0;
  if (type == TYPE_CUT && ncx > 0 && Sw > 0.0) {
    const double r[3] = {rs[0] / ncx, rs[1] / ncx, rs[2] / ncx};
    aw = Sw;
    n0 = Aw[0] / Sw; n1 = Aw[1] / Sw; n2 = Aw[2] / Sw;
    V += (r[0] * Aw[0] + r[1] * Aw[1] + r[2] * Aw[2]) / 3.0;
    r0 = G.x0 + i * G.dx + r[0];
    r1 = G.y0 + j * G.dy + r[1];
    r2 = G.z0 + k * G.dz + r[2];
  }
  G.type[t] = type;
  G.flags[t] = flags;
  G.sxm[t] = S[0]; G.sxp[t] = S[1]; G.sym[t] = S[2];
  G.syp[t] = S[3]; G.szm[t] = S[4]; G.szp[t] = S[5];
  G.aw[t] = aw; G.nwx[t] = n0; G.nwy[t] = n1; G.nwz[t] = n2;
  G.rwx[t] = r0; G.rwy[t] = r1; G.rwz[t] = r2;
  G.vbar[t] = type == TYPE_SOLID ? 0.0 : (type == TYPE_GAS ? G.dx * G.dy * G.dz : V);
}

// one hop across the largest face shared with a cell of the domain
__device__ inline bool hop3d(const Geo3D& G, int& i, int& j, int& k) {
  const int c = (k * G.ny + j) * G.nx + i;
  const double L[6] = {i + 1 < G.nx ? G.sxp[c] : 0.0, i > 0 ? G.sxm[c] : 0.0,
                       j + 1 < G.ny ? G.syp[c] : 0.0, j > 0 ? G.sym[c] : 0.0,
                       k + 1 < G.nz ? G.szp[c] : 0.0, k > 0 ? G.szm[c] : 0.0};
  double M = 0.0;
  for (int u = 0; u < 6; ++u) M = L[u] > M ? L[u] : M;
  if (!(M > 0.0)) return false;
  const double tie = M * (1.0 - 1e-12);
  int u = 0;
  while (L[u] < tie) ++u;
  switch (u) {
    case 0: i += 1; break;
    case 1: i -= 1; break;
    case 2: j += 1; break;
    case 3: j -= 1; break;
    case 4: k += 1; break;
    default: k -= 1; break;
  }
  return true;
}

__global__ void k_master3d(Geo3D G) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.ncell) return;
  if (G.type[c] == TYPE_SOLID) { G.master[c] = -1; return; }
  int i = c % G.nx, j = (c / G.nx) % G.ny, k = c / (G.nx * G.ny);
  int seen[kHopCap + 1];
  seen[0] = c;
  int hops = 0;
  bool bad = false;
  while (!(G.flags[(k * G.ny + j) * G.nx + i] & 1)) {
    if (hops == kHopCap || !hop3d(G, i, j, k)) { bad = true; break; }
    ++hops;
    const int nc = (k * G.ny + j) * G.nx + i;
    for (int h = 0; h < hops; ++h) bad |= seen[h] == nc;
    if (bad) break;
    seen[hops] = nc;
  }
  G.master[c] = (k * G.ny + j) * G.nx + i;
  if (bad) atomicOr(&G.counts[3], 1);
  if (G.flags[c] & 2) atomicOr(&G.counts[3], 2);
}

// Visits the cells of the window of half-width kHopCap around cell m in
// ascending cell order.
template <class F>
__device__ inline void for_window(const Geo3D& G, int m, F&& f) {
  const int i = m % G.nx, j = (m / G.nx) % G.ny, k = m / (G.nx * G.ny);
  for (int kk = max(k - kHopCap, 0); kk <= min(k + kHopCap, G.nz - 1); ++kk)
    for (int jj = max(j - kHopCap, 0); jj <= min(j + kHopCap, G.ny - 1); ++jj)
      for (int ii = max(i - kHopCap, 0); ii <= min(i + kHopCap, G.nx - 1); ++ii)
        f((kk * G.ny + jj) * G.nx + ii);
}

// control-volume volume and kind; a master that owns members touches a cut
// cell through a face (the last hop of a member's search crosses it)
__global__ void k_cv3d(Geo3D G) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.ncell) return;
  const int m = G.master[c];
  if (m < 0) { G.kind[c] = KIND_SOLID; G.vcv[c] = 0.0; return; }
  if (m != c) { G.kind[c] = KIND_MEMBER; G.vcv[c] = 0.0; return; }
  const int i = c % G.nx, j = (c / G.nx) % G.ny, k = c / (G.nx * G.ny);
  bool near_cut = false;
  for (int dk = -1; dk <= 1; ++dk)
    for (int dj = -1; dj <= 1; ++dj)
      for (int di = -1; di <= 1; ++di) {
        const int ii = i + di, jj = j + dj, kk = k + dk;
        if (ii >= 0 && jj >= 0 && kk >= 0 && ii < G.nx && jj < G.ny && kk < G.nz)
          near_cut |= G.type[(kk * G.ny + jj) * G.nx + ii] == TYPE_CUT;
      }
  double V = 0.0;
  int cnt = 0;
  if (!near_cut) {
    V = G.vbar[c];
    cnt = 1;
  } else {
    for_window(G, c, [&](int q) {
      if (G.master[q] == c) { V += G.vbar[q]; ++cnt; }
    });
  }
  G.vcv[c] = V;
  G.kind[c] = (G.type[c] == TYPE_GAS && cnt == 1) ? KIND_REGULAR : KIND_IRREGULAR;
  if (cnt > kMaxMembers) atomicOr(&G.counts[3], 4);
}

__device__ int block_scan(int v, int* sh, int* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const int add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const int incl = sh[t];
  *total = sh[blockDim.x - 1];
  __syncthreads();
  return incl - v;
}

// single-block deterministic compaction: irregular masters in ascending
// order, CSR of their members (ascending), population counts
__global__ void __launch_bounds__(1024) k_compact3d(Geo3D G) {
  __shared__ int sh[1024];
  const int t = threadIdx.x;
  const int per = (G.ncell + blockDim.x - 1) / blockDim.x;
  const int b = t * per, e = min(b + per, G.ncell);
  int nirr = 0, nmem = 0, nsol = 0;
  for (int u = b; u < e; ++u) {
    const int kd = G.kind[u];
    nirr += kd == KIND_IRREGULAR;
    nmem += kd == KIND_MEMBER;
    nsol += kd == KIND_SOLID;
  }
  int tot_irr, tot_mem, tot_sol;
  int off = block_scan(nirr, sh, &tot_irr);
  block_scan(nmem, sh, &tot_mem);
  block_scan(nsol, sh, &tot_sol);
  for (int u = b; u < e; ++u)
    if (G.kind[u] == KIND_IRREGULAR) G.irr[off++] = u;
  if (t == 0) { G.counts[0] = tot_irr; G.counts[1] = tot_mem; G.counts[2] = tot_sol; }
  __syncthreads();
  int carry = 0;
  for (int base = 0; base < tot_irr; base += blockDim.x) {
    const int q = base + t;
    int cnt = 0;
    if (q < tot_irr) {
      const int m = G.irr[q];
      for_window(G, m, [&](int c) { cnt += G.master[c] == m; });
    }
    int tot;
    const int ex = block_scan(cnt, sh, &tot);
    if (q < tot_irr) G.mptr[q] = carry + ex;
    carry += tot;
  }
  if (t == 0) G.mptr[tot_irr] = carry;
  __syncthreads();
  for (int q = t; q < tot_irr; q += blockDim.x) {
    const int m = G.irr[q];
    int w = G.mptr[q];
    for_window(G, m, [&](int c) {
      if (G.master[c] == m) G.mem[w++] = c;
    });
  }
}

// velocity nodes and the farfield table (3D Maxwellian, eq. MaxwellianTD)
__global__ void k_tables3d(Geo3D G, double vmin, double dv, double rho, double ux, double uy,
                           double uz, double T) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < G.N) G.vnode[p] = vmin + (p + 0.5) * dv;
  if (p >= G.nvel) return;
  const int N = G.N;
  const double vx = vmin + (p % N + 0.5) * dv, vy = vmin + ((p / N) % N + 0.5) * dv,
               vz = vmin + (p / (N * N) + 0.5) * dv;
  const double cx = vx - ux, cy = vy - uy, cz = vz - uz;
  G.ghost[p] = rho / pow(2.0 * M_PI * T, 1.5) * exp(-(cx * cx + cy * cy + cz * cz) / (2.0 * T));
}

}  // namespace

hipError_t build_geometry_3d(cc_ctx* ctx) {
  Geo3D& G = ctx->g3;
  hipStream_t s = ctx->stream;
  BodyDev B{};
  B.kind = ctx->body.kind;
  B.cx = ctx->body.center[0]; B.cy = ctx->body.center[1]; B.cz = ctx->body.center[2];
  B.a = ctx->body.axes[0];
  B.t_wall = ctx->body.t_wall;
  hipError_t e = hipMemsetAsync(G.counts, 0, 4 * sizeof(int), s);
  if (e != hipSuccess) return e;
  const long long nv = (long long)(G.nx + 1) * (G.ny + 1) * (G.nz + 1);
  const int nc = G.ncell;
  k_phi3d<<<(unsigned)((nv + 255) / 256), 256, 0, s>>>(G, B);
  k_cell3d<<<(nc + 255) / 256, 256, 0, s>>>(G);
  k_master3d<<<(nc + 255) / 256, 256, 0, s>>>(G);
  k_cv3d<<<(nc + 255) / 256, 256, 0, s>>>(G);
  k_compact3d<<<1, 1024, 0, s>>>(G);
  const double* in = ctx->cfg.inflow;
  const int nt = G.nvel > G.N ? G.nvel : G.N;
  k_tables3d<<<(nt + 255) / 256, 256, 0, s>>>(G, ctx->cfg.vmin, ctx->dv, in[0], in[1], in[2],
                                              in[3], in[4]);
  return hipGetLastError();
}

}  // namespace ccdvm
