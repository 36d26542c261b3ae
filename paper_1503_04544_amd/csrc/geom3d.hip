// Device construction of the 3D cut-cell geometry (Section 5, fixed body).
// The paper leaves the 3D geometry to the reader; the rules used here:
//   * vertex level set with the 1e-10 dx clamp, sign(0) = +1;
//   * per-cell faces, wall and volume as in cellgeom3d.h (the 2D
//     virtual-cell rule on each face's four vertices, a wall face that closes
//     the cell, the divergence theorem for the volume);
//   * master search: centre in gas when the mean of the 8 vertex values
//     exceeds 1e-12 dx, otherwise hop across the largest face shared with a
//     cell of the domain (ties within 1e-12 broken in the order x+, x-, y+,
//     y-, z+, z-), at most 4 hops, no revisits.
// Floating-point contraction is off in this file so that the tables are the
// correctly rounded evaluation of these formulas in the order written, which
// keeps tie decisions reproducible.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include "ccdvm_impl.h"

#pragma clang fp contract(off)

#include "cellgeom3d.h"

namespace ccdvm {
namespace {

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

__global__ void k_cell3d(Geo3D G) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= G.ncell) return;
  const int i = t % G.nx, j = (t / G.nx) % G.ny, k = t / (G.nx * G.ny);
  double qv[8];   // corner b at ((b >> 2) & 1, (b >> 1) & 1, b & 1)
  for (int b = 0; b < 8; ++b) qv[b] = vtx(G, i, j, k, (b >> 2) & 1, (b >> 1) & 1, b & 1);
  const double h[3] = {G.dx, G.dy, G.dz};
  CellGeo3 c;
  cell_geometry_3d(qv, h, 1e-12 * G.dx, c);
  G.type[t] = c.type;
  G.flags[t] = c.flags;
  G.sxm[t] = c.S[0]; G.sxp[t] = c.S[1]; G.sym[t] = c.S[2];
  G.syp[t] = c.S[3]; G.szm[t] = c.S[4]; G.szp[t] = c.S[5];
  G.aw[t] = c.aw; G.nwx[t] = c.n[0]; G.nwy[t] = c.n[1]; G.nwz[t] = c.n[2];
  if (c.aw > 0.0) {
    G.rwx[t] = G.x0 + i * G.dx + c.r[0];
    G.rwy[t] = G.y0 + j * G.dy + c.r[1];
    G.rwz[t] = G.z0 + k * G.dz + c.r[2];
  } else {
    G.rwx[t] = 0.0; G.rwy[t] = 0.0; G.rwz[t] = 0.0;
  }
  G.vbar[t] = c.vbar;
}

// One hop across the largest face shared with a cell of the domain.  Faces
// are ranked x+, x-, y+, y-, z+, z- (direction u: axis u / 2, upward for
// even u); the first one within a relative 1e-12 of the largest wins.
__device__ inline bool hop3d(const Geo3D& G, int& i, int& j, int& k) {
  const int c = (k * G.ny + j) * G.nx + i;
  int pos[3] = {i, j, k};
  const int ext[3] = {G.nx, G.ny, G.nz};
  const double* area[6] = {G.sxp, G.sxm, G.syp, G.sym, G.szp, G.szm};
  double len[6], best = 0.0;
  for (int u = 0; u < 6; ++u) {
    const int nb = pos[u >> 1] + ((u & 1) ? -1 : 1);
    len[u] = (nb >= 0 && nb < ext[u >> 1]) ? area[u][c] : 0.0;
    best = fmax(best, len[u]);
  }
  if (!(best > 0.0)) return false;
  int u = 0;
  while (len[u] < best * (1.0 - 1e-12)) ++u;
  pos[u >> 1] += (u & 1) ? -1 : 1;
  i = pos[0]; j = pos[1]; k = pos[2];
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
  int off = block_scan_excl(nirr, sh, &tot_irr);
  block_scan_excl(nmem, sh, &tot_mem);
  block_scan_excl(nsol, sh, &tot_sol);
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
    const int ex = block_scan_excl(cnt, sh, &tot);
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

// Outflow rate of eq. (phiCFL), in its 3D form (six faces and the wall),
// of each cut or merged control volume divided by its volume, maximised over
// the velocity grid: convex in v, so the largest value is at one of the
// eight corner nodes.  Fixed wall (u_w = 0).
__global__ void k_cfl3d(Geo3D G, int nirr, double vlo, double vhi, unsigned long long* out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nirr) return;
  const int m = G.irr[q];
  double best = 0.0;
  for (int corner = 0; corner < 8; ++corner) {
    const double v1 = (corner & 1) ? vhi : vlo, v2 = (corner & 2) ? vhi : vlo, v3 = (corner & 4) ? vhi : vlo;
    double phi = 0.0;
    for (int e = G.mptr[q]; e < G.mptr[q + 1]; ++e) {
      const int k = G.mem[e];
      phi += G.sxp[k] * fmax(v1, 0.0) - G.sxm[k] * fmin(v1, 0.0) + G.syp[k] * fmax(v2, 0.0) -
             G.sym[k] * fmin(v2, 0.0) + G.szp[k] * fmax(v3, 0.0) - G.szm[k] * fmin(v3, 0.0);
      if (G.aw[k] > 0.0) phi += G.aw[k] * fmax(v1 * G.nwx[k] + v2 * G.nwy[k] + v3 * G.nwz[k], 0.0);
    }
    best = fmax(best, phi / G.vcv[m]);
  }
  atomicMax(out, (unsigned long long)__double_as_longlong(best));
}

}  // namespace

hipError_t cfl_rate_3d(cc_ctx* ctx, double vlo, double vhi, double* rate) {
  unsigned long long* word = reinterpret_cast<unsigned long long*>(ctx->s.red);
  hipError_t e = hipMemsetAsync(word, 0, sizeof(unsigned long long), ctx->stream);
  if (e != hipSuccess) return e;
  if (ctx->n_irr > 0)
    k_cfl3d<<<(ctx->n_irr + 127) / 128, 128, 0, ctx->stream>>>(ctx->g3, ctx->n_irr, vlo, vhi, word);
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

hipError_t build_geometry_3d(cc_ctx* ctx) {
  Geo3D& G = ctx->g3;
  hipStream_t s = ctx->stream;
  BodyDev B{};
  B.kind = ctx->body.kind;
  B.cx = ctx->body.center[0]; B.cy = ctx->body.center[1]; B.cz = ctx->body.center[2];
  B.a = ctx->body.axes[0]; B.b = ctx->body.axes[1]; B.c = ctx->body.axes[2];
  B.theta = ctx->body.theta;
  B.ct = cos(B.theta); B.st = sin(B.theta);
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
