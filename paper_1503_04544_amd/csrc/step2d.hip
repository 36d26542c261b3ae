// One explicit time step of the 2D reduced model (f, g) on gfx950.
//
// Scheme (Section 3.3): for every control volume, the first-order explicit
// update (eq. ExSchemeDD) with upwind fluxes on its Cartesian and wall edges
// (eq. FluxDD), the diffuse wall distribution with the density that cancels
// the net mass flux (eq. BoundaryDDv), the BGK relaxation toward the
// Maxwellian of the discrete moments (eqs. MacroscopicDDv, BGKDD), and the
// redistribution to the merged virtual cells (eq. UpdateDD).
//
// Work split.  Gas cells whose control volume is the cell itself (all but a
// fraction of a percent of the cells) go through k_regular2d, a streaming
// stencil: per (cell, velocity) it reads the cell, its upwind neighbour in x
// and in y, and writes the new (f, g).  The moments that the relaxation needs
// are those of the state being advanced; they were produced by the epilogue
// of the previous step (the wave that writes a cell's new values also sums
// its moments), so the kernel never waits for a reduction before streaming.
// Control volumes that are cut or own merged cells go through k_cut2d, one
// wave each.  Both kernels read state `in` and write state `out`.
//
// Layout: double2 state[c][p] = {f, g}; p = p2*N + p1; lane l of a wave
// handles velocities p = 64*k + l, so a wave load is 1 KiB contiguous.
#include <hip/hip_runtime.h>

#include <math.h>

#include "ccdvm_impl.h"

namespace ccdvm {
namespace {

constexpr int kWave = 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline double vnode(double vmin, double dv, int idx) { return vmin + (idx + 0.5) * dv; }

struct StepParams {
  double vmin, dv, w;     // velocity box, node spacing, weight dv^2
  double dt;
  double tau_coef;        // tau = tau_coef / rho; 0 = no collisions
  double t_wall;
  int moving;
  int write_state;        // 0: cut-cell kernel only computes the wall forces
};

// ---------------------------------------------------------------------
// Regular gas cells: fused transport + relaxation + moments of the result.
// NCH = number of 64-velocity chunks per cell (ceil(N^2 / 64)).
// ---------------------------------------------------------------------
template <int NCH>
__global__ void __launch_bounds__(256) k_regular2d(Geo2D G, const double2* __restrict__ in,
                                                   double2* __restrict__ out,
                                                   double* __restrict__ mom, StepParams P) {
  const int lane = threadIdx.x & (kWave - 1);
  const int c = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (c >= G.ncell) return;
  if (G.kind[c] != KIND_REGULAR) return;
  const int N = G.N, nvel = G.nvel, nx = G.nx;
  const int i = c % nx, j = c / nx;
  const double rho = mom[4 * c + 0], ux = mom[4 * c + 1], uy = mom[4 * c + 2], T = mom[4 * c + 3];
  const double inv2T = 0.5 / T;
  const double A = rho / (2.0 * M_PI * T);
  const double dtau = P.tau_coef > 0.0 ? P.dt * rho / P.tau_coef : 0.0;
  // separable Maxwellian: lane l < N holds exp(-(v_l - u)^2 / 2T) per axis
  double tx = 0.0, ty = 0.0;
  if (lane < N) {
    double v = vnode(P.vmin, P.dv, lane);
    tx = exp(-(v - ux) * (v - ux) * inv2T);
    ty = exp(-(v - uy) * (v - uy) * inv2T);
  }
  const double S = G.dx * G.dy;
  const double cxf = P.dt / S * G.dy, cyf = P.dt / S * G.dx;
  const double2* incell = in + (size_t)c * nvel;
  double2* outcell = out + (size_t)c * nvel;
  double sr = 0.0, smx = 0.0, smy = 0.0, se = 0.0;
#pragma unroll 4
  for (int k = 0; k < NCH; ++k) {
    const int p = k * kWave + lane;
    const bool ok = p < nvel;
    const int pp = ok ? p : 0;
    const int p1 = pp % N, p2 = pp / N;
    const double vx = vnode(P.vmin, P.dv, p1), vy = vnode(P.vmin, P.dv, p2);
    const double2 own = incell[pp];
    double2 xu, yu;
    if (vx > 0.0) xu = i > 0 ? incell[pp - (ptrdiff_t)nvel] : G.ghost[pp];
    else xu = i + 1 < nx ? incell[pp + (ptrdiff_t)nvel] : G.ghost[pp];
    if (vy > 0.0) yu = j > 0 ? incell[pp - (ptrdiff_t)nx * nvel] : G.ghost[pp];
    else yu = j + 1 < G.ny ? incell[pp + (ptrdiff_t)nx * nvel] : G.ghost[pp];
    const double ax = cxf * fabs(vx), ay = cyf * fabs(vy);
    const double E = A * __shfl(tx, p1, kWave) * __shfl(ty, p2, kWave);
    double fn = own.x - ax * (own.x - xu.x) - ay * (own.x - yu.x) + dtau * (E - own.x);
    double gn = own.y - ax * (own.y - xu.y) - ay * (own.y - yu.y) + dtau * (0.5 * T * E - own.y);
    if (ok) {
      outcell[p] = make_double2(fn, gn);
      sr += fn;
      smx += vx * fn;
      smy += vy * fn;
      se += 0.5 * (vx * vx + vy * vy) * fn + gn;
    }
  }
  sr = wave_sum(sr); smx = wave_sum(smx); smy = wave_sum(smy); se = wave_sum(se);
  if (lane == 0) {
    double r = sr * P.w, mx = smx * P.w / r, my = smy * P.w / r, e = se * P.w;
    mom[4 * c + 0] = r;
    mom[4 * c + 1] = mx;
    mom[4 * c + 2] = my;
    mom[4 * c + 3] = (2.0 * e / r - (mx * mx + my * my)) / 3.0;
  }
}

__device__ inline void wall_velocity(const double* body, double rx, double ry, double* uwx,
                                     double* uwy) {
  // u_w = u_sol + (r - c)^perp omega, a^perp = (-a_y, a_x)
  *uwx = body[3] - (ry - body[1]) * body[5];
  *uwy = body[4] + (rx - body[0]) * body[5];
}

__device__ inline double maxw_wall(double vx, double vy, double uwx, double uwy, double Tw) {
  double ex = vx - uwx, ey = vy - uwy;
  return exp(-(ex * ex + ey * ey) / (2.0 * Tw)) / (2.0 * M_PI * Tw);
}

// ---------------------------------------------------------------------
// Control volumes that are cut or own merged cells: one wave each.
// fslot[q] receives (Fx, Fy, torque) of the wall edges of the control volume
// from the state being advanced (eqs. StressTensorDD, eq-force, eq-torque).
// ---------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_cut2d(Geo2D G, const double2* __restrict__ in,
                                              double2* __restrict__ out,
                                              double* __restrict__ mom,
                                              double* __restrict__ fslot,
                                              const double* __restrict__ body, StepParams P) {
  const int q = blockIdx.x;
  const int lane = threadIdx.x;
  const int m = G.irr[q];
  const int b = G.mptr[q], e = G.mptr[q + 1];
  const int nm = e - b;
  const int N = G.N, nvel = G.nvel, nx = G.nx, ny = G.ny;
  const double rho = mom[4 * m + 0], ux = mom[4 * m + 1], uy = mom[4 * m + 2], T = mom[4 * m + 3];
  const double inv2T = 0.5 / T, A = rho / (2.0 * M_PI * T);
  const double dtau = P.tau_coef > 0.0 ? P.dt * rho / P.tau_coef : 0.0;
  const double S = G.scv[m];
  const double2* own = in + (size_t)m * nvel;
  const double Tw = P.t_wall;
  // wall density of every wall edge of the control volume
  double phiw[kMaxMembers], uwx[kMaxMembers], uwy[kMaxMembers];
  for (int t = 0; t < nm; ++t) {
    const int k = G.mem[b + t];
    phiw[t] = 0.0; uwx[t] = 0.0; uwy[t] = 0.0;
    if (!(G.lw[k] > 0.0)) continue;
    wall_velocity(body, G.rwx[k], G.rwy[k], &uwx[t], &uwy[t]);
    const double nwx = G.nwx[k], nwy = G.nwy[k];
    double num = 0.0, den = 0.0;
    for (int p = lane; p < nvel; p += kWave) {
      const double vx = vnode(P.vmin, P.dv, p % N), vy = vnode(P.vmin, P.dv, p / N);
      const double cn = (vx - uwx[t]) * nwx + (vy - uwy[t]) * nwy;
      if (cn > 0.0) num += cn * own[p].x;
      else if (cn < 0.0) den += cn * maxw_wall(vx, vy, uwx[t], uwy[t], Tw);
    }
    num = wave_sum(num);
    den = wave_sum(den);
    phiw[t] = den != 0.0 ? -num / den : 0.0;
  }
  double sx[kMaxMembers], sy[kMaxMembers];
  for (int t = 0; t < kMaxMembers; ++t) { sx[t] = 0.0; sy[t] = 0.0; }
  double sr = 0.0, smx = 0.0, smy = 0.0, se = 0.0;
  for (int p = lane; p < nvel; p += kWave) {
    const int p1 = p % N, p2 = p / N;
    const double vx = vnode(P.vmin, P.dv, p1), vy = vnode(P.vmin, P.dv, p2);
    const double vxm = fmin(vx, 0.0), vxp = fmax(vx, 0.0);
    const double vym = fmin(vy, 0.0), vyp = fmax(vy, 0.0);
    const double2 o = own[p];
    double Rf = 0.0, Rg = 0.0;
    for (int t = 0; t < nm; ++t) {
      const int k = G.mem[b + t];
      const int i = k % nx, j = k / nx;
      const double Lr = G.lxp[k], Ll = G.lxm[k], Lt = G.lyp[k], Lb = G.lym[k];
      if (Lr > 0.0) {
        double2 nb = i + 1 < nx ? in[(size_t)(k + 1) * nvel + p] : G.ghost[p];
        Rf += Lr * (vxm * nb.x + vxp * o.x);
        Rg += Lr * (vxm * nb.y + vxp * o.y);
      }
      if (Ll > 0.0) {
        double2 nb = i > 0 ? in[(size_t)(k - 1) * nvel + p] : G.ghost[p];
        Rf -= Ll * (vxm * o.x + vxp * nb.x);
        Rg -= Ll * (vxm * o.y + vxp * nb.y);
      }
      if (Lt > 0.0) {
        double2 nb = j + 1 < ny ? in[(size_t)(k + nx) * nvel + p] : G.ghost[p];
        Rf += Lt * (vym * nb.x + vyp * o.x);
        Rg += Lt * (vym * nb.y + vyp * o.y);
      }
      if (Lb > 0.0) {
        double2 nb = j > 0 ? in[(size_t)(k - nx) * nvel + p] : G.ghost[p];
        Rf -= Lb * (vym * o.x + vyp * nb.x);
        Rg -= Lb * (vym * o.y + vyp * nb.y);
      }
      const double Lw = G.lw[k];
      if (Lw > 0.0) {
        const double cx_ = vx - uwx[t], cy_ = vy - uwy[t];
        const double cn = cx_ * G.nwx[k] + cy_ * G.nwy[k];
        const double Mw = maxw_wall(vx, vy, uwx[t], uwy[t], Tw);
        const double fw = phiw[t] * Mw, gw = phiw[t] * 0.5 * Tw * Mw;
        Rf += Lw * (fmin(cn, 0.0) * fw + fmax(cn, 0.0) * o.x);
        Rg += Lw * (fmin(cn, 0.0) * gw + fmax(cn, 0.0) * o.y);
        const double fv = cn < 0.0 ? fw : (cn > 0.0 ? o.x : 0.0);
        sx[t] += cx_ * cn * fv;
        sy[t] += cy_ * cn * fv;
      }
    }
    double E = 0.0;
    if (dtau != 0.0) {
      const double ex = vx - ux, ey = vy - uy;
      E = A * exp(-ex * ex * inv2T) * exp(-ey * ey * inv2T);
    }
    const double fn = o.x - P.dt / S * Rf + dtau * (E - o.x);
    const double gn = o.y - P.dt / S * Rg + dtau * (0.5 * T * E - o.y);
    if (P.write_state)
      for (int t = 0; t < nm; ++t) out[(size_t)G.mem[b + t] * nvel + p] = make_double2(fn, gn);
    sr += fn; smx += vx * fn; smy += vy * fn;
    se += 0.5 * (vx * vx + vy * vy) * fn + gn;
  }
  double Fx = 0.0, Fy = 0.0, Tq = 0.0;
  for (int t = 0; t < nm; ++t) {
    const int k = G.mem[b + t];
    const double ax = wave_sum(sx[t]) * P.w, ay = wave_sum(sy[t]) * P.w;
    if (G.lw[k] > 0.0) {
      Fx += ax * G.lw[k];
      Fy += ay * G.lw[k];
      Tq += ((G.rwx[k] - body[0]) * ay - (G.rwy[k] - body[1]) * ax) * G.lw[k];
    }
  }
  sr = wave_sum(sr); smx = wave_sum(smx); smy = wave_sum(smy); se = wave_sum(se);
  if (lane == 0) {
    double r = sr * P.w, mx = smx * P.w / r, my = smy * P.w / r, en = se * P.w;
    double Tn = (2.0 * en / r - (mx * mx + my * my)) / 3.0;
    if (P.write_state)
      for (int t = 0; t < nm; ++t) {
        const int k = G.mem[b + t];
        mom[4 * k + 0] = r; mom[4 * k + 1] = mx; mom[4 * k + 2] = my; mom[4 * k + 3] = Tn;
      }
    fslot[3 * q + 0] = Fx;
    fslot[3 * q + 1] = Fy;
    fslot[3 * q + 2] = Tq;
  }
}

// ---------------------------------------------------------------------
// Merge (eq. FusionDD) of control volumes with several members, in place,
// followed by the moments of the merged value.
// ---------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_merge2d(Geo2D G, double2* __restrict__ st,
                                                double* __restrict__ mom, StepParams P) {
  const int q = blockIdx.x, lane = threadIdx.x;
  const int m = G.irr[q];
  const int b = G.mptr[q], e = G.mptr[q + 1];
  const int N = G.N, nvel = G.nvel;
  const double S = G.scv[m];
  double sr = 0.0, smx = 0.0, smy = 0.0, se = 0.0;
  for (int p = lane; p < nvel; p += kWave) {
    double af = 0.0, ag = 0.0;
    if (e - b > 1) {
      for (int t = b; t < e; ++t) {
        const int k = G.mem[t];
        const double2 v = st[(size_t)k * nvel + p];
        af += G.sbar[k] * v.x;
        ag += G.sbar[k] * v.y;
      }
      af /= S; ag /= S;
      for (int t = b; t < e; ++t) st[(size_t)G.mem[t] * nvel + p] = make_double2(af, ag);
    } else {
      const double2 v = st[(size_t)m * nvel + p];
      af = v.x; ag = v.y;
    }
    const double vx = vnode(P.vmin, P.dv, p % N), vy = vnode(P.vmin, P.dv, p / N);
    sr += af; smx += vx * af; smy += vy * af;
    se += 0.5 * (vx * vx + vy * vy) * af + ag;
  }
  sr = wave_sum(sr); smx = wave_sum(smx); smy = wave_sum(smy); se = wave_sum(se);
  if (lane == 0) {
    double r = sr * P.w, mx = smx * P.w / r, my = smy * P.w / r, en = se * P.w;
    double Tn = (2.0 * en / r - (mx * mx + my * my)) / 3.0;
    for (int t = b; t < e; ++t) {
      const int k = G.mem[t];
      mom[4 * k + 0] = r; mom[4 * k + 1] = mx; mom[4 * k + 2] = my; mom[4 * k + 3] = Tn;
    }
  }
}

// moments (rho, u, T) of every non-solid cell, one wave per cell
__global__ void __launch_bounds__(256) k_mom2d(Geo2D G, const double2* __restrict__ st,
                                               double* __restrict__ mom, StepParams P) {
  const int lane = threadIdx.x & (kWave - 1);
  const int c = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (c >= G.ncell || G.kind[c] == KIND_SOLID) return;
  const int N = G.N, nvel = G.nvel;
  double sr = 0.0, smx = 0.0, smy = 0.0, se = 0.0;
  for (int p = lane; p < nvel; p += kWave) {
    const double2 v = st[(size_t)c * nvel + p];
    const double vx = vnode(P.vmin, P.dv, p % N), vy = vnode(P.vmin, P.dv, p / N);
    sr += v.x; smx += vx * v.x; smy += vy * v.x;
    se += 0.5 * (vx * vx + vy * vy) * v.x + v.y;
  }
  sr = wave_sum(sr); smx = wave_sum(smx); smy = wave_sum(smy); se = wave_sum(se);
  if (lane == 0) {
    double r = sr * P.w, mx = smx * P.w / r, my = smy * P.w / r, en = se * P.w;
    mom[4 * c + 0] = r; mom[4 * c + 1] = mx; mom[4 * c + 2] = my;
    mom[4 * c + 3] = (2.0 * en / r - (mx * mx + my * my)) / 3.0;
  }
}

// full moments for output: rho, ux, uy, T, Sxx, Sxy, Syy, qx, qy
__global__ void __launch_bounds__(256) k_momout2d(Geo2D G, const double2* __restrict__ st,
                                                  double* __restrict__ out, StepParams P) {
  const int lane = threadIdx.x & (kWave - 1);
  const int c = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (c >= G.ncell) return;
  double* o = out + (size_t)9 * c;
  if (G.kind[c] == KIND_SOLID) {
    if (lane < 9) o[lane] = 0.0;
    return;
  }
  const int N = G.N, nvel = G.nvel;
  double sr = 0.0, smx = 0.0, smy = 0.0, se = 0.0;
  for (int p = lane; p < nvel; p += kWave) {
    const double2 v = st[(size_t)c * nvel + p];
    const double vx = vnode(P.vmin, P.dv, p % N), vy = vnode(P.vmin, P.dv, p / N);
    sr += v.x; smx += vx * v.x; smy += vy * v.x;
    se += 0.5 * (vx * vx + vy * vy) * v.x + v.y;
  }
  sr = wave_sum(sr); smx = wave_sum(smx); smy = wave_sum(smy); se = wave_sum(se);
  const double r = sr * P.w, ux = smx * P.w / r, uy = smy * P.w / r, en = se * P.w;
  const double T = (2.0 * en / r - (ux * ux + uy * uy)) / 3.0;
  double a = 0, bxy = 0, cyy = 0, qx = 0, qy = 0;
  for (int p = lane; p < nvel; p += kWave) {
    const double2 v = st[(size_t)c * nvel + p];
    const double cx = vnode(P.vmin, P.dv, p % N) - ux, cy = vnode(P.vmin, P.dv, p / N) - uy;
    a += cx * cx * v.x; bxy += cx * cy * v.x; cyy += cy * cy * v.x;
    const double h = 0.5 * (cx * cx + cy * cy) * v.x + v.y;
    qx += cx * h; qy += cy * h;
  }
  a = wave_sum(a); bxy = wave_sum(bxy); cyy = wave_sum(cyy); qx = wave_sum(qx); qy = wave_sum(qy);
  if (lane == 0) {
    o[0] = r; o[1] = ux; o[2] = uy; o[3] = T;
    o[4] = a * P.w; o[5] = bxy * P.w; o[6] = cyy * P.w; o[7] = qx * P.w; o[8] = qy * P.w;
  }
}

__global__ void k_init2d(Geo2D G, double2* __restrict__ st) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t tot = (size_t)G.ncell * G.nvel;
  if (t >= tot) return;
  int c = (int)(t / G.nvel), p = (int)(t % G.nvel);
  st[t] = G.kind[c] == KIND_SOLID ? make_double2(0.0, 0.0) : G.ghost[p];
}

__global__ void k_load2d(Geo2D G, double2* __restrict__ st, const double* __restrict__ f,
                         const double* __restrict__ g) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t tot = (size_t)G.ncell * G.nvel;
  if (t >= tot) return;
  int c = (int)(t / G.nvel);
  st[t] = G.kind[c] == KIND_SOLID ? make_double2(0.0, 0.0) : make_double2(f[t], g[t]);
}

__global__ void k_store2d(Geo2D G, const double2* __restrict__ st, double* __restrict__ f,
                          double* __restrict__ g) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t tot = (size_t)G.ncell * G.nvel;
  if (t >= tot) return;
  double2 v = st[t];
  f[t] = v.x;
  if (g) g[t] = v.y;
}

// Deterministic reduction of the per-control-volume forces and of the mass
// sum_m S_m rho_m.  Every block sums a fixed slice; the last block to finish
// adds the block partials in block order.
constexpr int kRedBlocks = 128;

__global__ void __launch_bounds__(256) k_reduce2d(Geo2D G, const double* __restrict__ mom,
                                                  const double* __restrict__ fslot,
                                                  double* __restrict__ red,
                                                  unsigned int* __restrict__ ticket,
                                                  double* force_row, double* mass_row) {
  __shared__ double sh[4][256];
  const int t = threadIdx.x;
  const int nb = gridDim.x;
  const int chunk = (G.ncell + nb - 1) / nb;
  const int c0 = blockIdx.x * chunk, c1 = min(c0 + chunk, G.ncell);
  double ms = 0.0;
  for (int c = c0 + t; c < c1; c += blockDim.x) {
    const int k = G.kind[c];
    if (k == KIND_REGULAR || k == KIND_IRREGULAR) ms += G.scv[c] * mom[4 * c];
  }
  const int nirr = G.counts[0];
  const int qchunk = (nirr + nb - 1) / nb;
  const int q0 = blockIdx.x * qchunk, q1 = min(q0 + qchunk, nirr);
  double fx = 0.0, fy = 0.0, tq = 0.0;
  for (int q = q0 + t; q < q1; q += blockDim.x) {
    fx += fslot[3 * q]; fy += fslot[3 * q + 1]; tq += fslot[3 * q + 2];
  }
  sh[0][t] = fx; sh[1][t] = fy; sh[2][t] = tq; sh[3][t] = ms;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s)
      for (int r = 0; r < 4; ++r) sh[r][t] += sh[r][t + s];
    __syncthreads();
  }
  __shared__ bool last;
  if (t == 0) {
    for (int r = 0; r < 4; ++r) red[4 * blockIdx.x + r] = sh[r][0];
    __threadfence();
    unsigned int prev = atomicAdd(ticket, 1u);
    last = prev == (unsigned int)nb - 1;
  }
  __syncthreads();
  if (last && t == 0) {
    __threadfence();
    double acc[4] = {0, 0, 0, 0};
    for (int b = 0; b < nb; ++b)
      for (int r = 0; r < 4; ++r) acc[r] += red[4 * b + r];
    if (force_row) { force_row[0] = acc[0]; force_row[1] = acc[1]; force_row[2] = acc[2]; }
    if (mass_row) mass_row[0] = acc[3];
    *ticket = 0u;
  }
}

StepParams params2d(const cc_ctx* ctx) {
  StepParams P;
  P.vmin = ctx->cfg.vmin;
  P.dv = ctx->dv;
  P.w = ctx->dv * ctx->dv;
  P.dt = ctx->dt;
  P.tau_coef = ctx->cfg.kn > 0.0 ? sqrt(M_PI) / 2.0 * ctx->cfg.kn * ctx->cfg.lref / sqrt(2.0) : 0.0;
  P.t_wall = ctx->body.t_wall;
  P.moving = ctx->body.motion != CC_MOTION_FIXED && ctx->body.kind != CC_BODY_NONE;
  P.write_state = 1;
  return P;
}

template <int NCH>
void launch_regular(const cc_ctx* ctx, const double2* in, double2* out, double* mom,
                    const StepParams& P) {
  const int cells_per_block = 4;
  dim3 grid((ctx->ncell + cells_per_block - 1) / cells_per_block);
  k_regular2d<NCH><<<grid, 256, 0, ctx->stream>>>(ctx->g2, in, out, mom, P);
}

typedef void (*regular_fn)(const cc_ctx*, const double2*, double2*, double*, const StepParams&);

regular_fn pick_regular(int nch) {
  switch (nch) {
    case 1: return launch_regular<1>;
    case 2: return launch_regular<2>;
    case 3: return launch_regular<3>;
    case 4: return launch_regular<4>;
    case 5: return launch_regular<5>;
    case 6: return launch_regular<6>;
    case 7: return launch_regular<7>;
    case 8: return launch_regular<8>;
    case 9: return launch_regular<9>;
    case 10: return launch_regular<10>;
    case 12: return launch_regular<12>;
    case 16: return launch_regular<16>;
    case 20: return launch_regular<20>;
    case 25: return launch_regular<25>;
    case 32: return launch_regular<32>;
    case 36: return launch_regular<36>;
    case 49: return launch_regular<49>;
    case 64: return launch_regular<64>;
    default: return nullptr;
  }
}

}  // namespace

bool regular_supported_2d(int nvel) { return pick_regular((nvel + 63) / 64) != nullptr; }

hipError_t launch_force_only_2d(cc_ctx* ctx, double* out4) {
  StepParams P = params2d(ctx);
  P.write_state = 0;
  const double2* in = (const double2*)ctx->state[ctx->cur];
  if (ctx->n_irr > 0)
    k_cut2d<<<ctx->n_irr, 64, 0, ctx->stream>>>(ctx->g2, in, (double2*)ctx->state[1 - ctx->cur],
                                                 ctx->s.mom, ctx->s.fslot, ctx->s.body, P);
  k_reduce2d<<<kRedBlocks, 256, 0, ctx->stream>>>(
      ctx->g2, ctx->s.mom, ctx->s.fslot, ctx->s.red,
      reinterpret_cast<unsigned int*>(ctx->s.red + 4 * kRedBlocks), out4, out4 + 3);
  return hipGetLastError();
}

hipError_t launch_init_maxwellian_2d(cc_ctx* ctx) {
  size_t tot = (size_t)ctx->ncell * ctx->nvel;
  k_init2d<<<(unsigned)((tot + 255) / 256), 256, 0, ctx->stream>>>(
      ctx->g2, (double2*)ctx->state[ctx->cur]);
  return hipGetLastError();
}

hipError_t launch_load_state_2d(cc_ctx* ctx, const double* f, const double* g) {
  size_t tot = (size_t)ctx->ncell * ctx->nvel;
  k_load2d<<<(unsigned)((tot + 255) / 256), 256, 0, ctx->stream>>>(
      ctx->g2, (double2*)ctx->state[ctx->cur], f, g);
  return hipGetLastError();
}

hipError_t launch_store_state_2d(const cc_ctx* ctx, double* f, double* g) {
  size_t tot = (size_t)ctx->ncell * ctx->nvel;
  k_store2d<<<(unsigned)((tot + 255) / 256), 256, 0, ctx->stream>>>(
      ctx->g2, (const double2*)ctx->state[ctx->cur], f, g);
  return hipGetLastError();
}

hipError_t launch_merge_2d(cc_ctx* ctx) {
  if (ctx->n_irr == 0) return hipSuccess;
  StepParams P = params2d(ctx);
  prof_begin(ctx, 3);
  k_merge2d<<<ctx->n_irr, 64, 0, ctx->stream>>>(ctx->g2, (double2*)ctx->state[ctx->cur],
                                                 ctx->s.mom, P);
  prof_end(ctx, 3);
  return hipGetLastError();
}

hipError_t launch_moments_all_2d(cc_ctx* ctx) {
  StepParams P = params2d(ctx);
  k_mom2d<<<(ctx->ncell + 3) / 4, 256, 0, ctx->stream>>>(
      ctx->g2, (const double2*)ctx->state[ctx->cur], ctx->s.mom, P);
  return hipGetLastError();
}

hipError_t launch_moments_out_2d(cc_ctx* ctx, double* out) {
  StepParams P = params2d(ctx);
  k_momout2d<<<(ctx->ncell + 3) / 4, 256, 0, ctx->stream>>>(
      ctx->g2, (const double2*)ctx->state[ctx->cur], out, P);
  return hipGetLastError();
}

// mass of the current state into mass_row (no force)
hipError_t launch_mass_2d(cc_ctx* ctx, double* mass_row) {
  k_reduce2d<<<kRedBlocks, 256, 0, ctx->stream>>>(
      ctx->g2, ctx->s.mom, ctx->s.fslot, ctx->s.red,
      reinterpret_cast<unsigned int*>(ctx->s.red + 4 * kRedBlocks), nullptr, mass_row);
  return hipGetLastError();
}

// One step: state[cur] -> state[1-cur].  force_row (nullable) receives the
// force and torque of the state at t^n; mass_row (nullable) the mass of the
// state at t^{n+1}.
hipError_t launch_step_2d(cc_ctx* ctx, double* force_row, double* mass_row) {
  StepParams P = params2d(ctx);
  const double2* in = (const double2*)ctx->state[ctx->cur];
  double2* out = (double2*)ctx->state[1 - ctx->cur];
  int nch = (ctx->nvel + 63) / 64;
  regular_fn fn = pick_regular(nch);
  if (!fn) return hipErrorInvalidValue;
  prof_begin(ctx, 0);
  fn(ctx, in, out, ctx->s.mom, P);
  prof_end(ctx, 0);
  if (ctx->n_irr > 0) {
    prof_begin(ctx, 1);
    k_cut2d<<<ctx->n_irr, 64, 0, ctx->stream>>>(ctx->g2, in, out, ctx->s.mom, ctx->s.fslot,
                                                 ctx->s.body, P);
    prof_end(ctx, 1);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (force_row || mass_row) {
    prof_begin(ctx, 2);
    k_reduce2d<<<kRedBlocks, 256, 0, ctx->stream>>>(
        ctx->g2, ctx->s.mom, ctx->s.fslot, ctx->s.red,
        reinterpret_cast<unsigned int*>(ctx->s.red + 4 * kRedBlocks), force_row, mass_row);
    prof_end(ctx, 2);
    e = hipGetLastError();
  }
  ctx->cur = 1 - ctx->cur;
  return e;
}


}  // namespace ccdvm
