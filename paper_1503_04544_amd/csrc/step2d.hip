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
#include <string.h>

#include <vector>

#include "ccdvm_impl.h"
#include "equilibrium.h"

namespace ccdvm {
namespace {

constexpr int kWave = 64;

__device__ inline double wave_sum(double v) { return wave_allsum(v); }

__device__ inline double vnode(double vmin, double dv, int idx) { return vmin + (idx + 0.5) * dv; }

struct StepParams {
  double vmin, dv, w;     // velocity box, node spacing, weight dv^2
  double dt;
  double tau_coef;        // tau = tau_coef / rho; 0 = no collisions
  double t_wall;
  int moving;
  int write_state;        // 0: cut-cell kernel only computes the wall forces
  int shakhov;            // relaxation toward the Shakhov equilibria (eq. ShakhovDD)
  int implicit;           // semi-implicit step: the cut-cell kernel transports only
  double sk_coef;         // (1 - Pr)/5
};

__device__ inline void wall_velocity(const double* body, double rx, double ry, double* uwx,
                                     double* uwy) {
  // u_w = u_sol + (r - c)^perp omega, a^perp = (-a_y, a_x)
  *uwx = body[3] - (ry - body[1]) * body[5];
  *uwy = body[4] + (rx - body[0]) * body[5];
}

constexpr int kMaxN2 = 64;  // largest number of velocity nodes per axis

// Velocity sums of one control volume's (f, g), from which eq.
// (MacroscopicDDv) gives rho, u, T and, with SK, the heat flux.  q is
// expanded in sums about v = 0 so that one pass over the values suffices:
//   q = 1/2 [S3 - 2 S2 u - u tr S2 + 2 rho |u|^2 u] + G1 - u G0,
// S2 = sum v v^T f, S3 = sum |v|^2 v f, G1 = sum v g, G0 = sum g.
template <bool SK>
struct Sums2 {
  double r = 0.0, mx = 0.0, my = 0.0, e = 0.0;
  double xx = 0.0, xy = 0.0, yy = 0.0, x3 = 0.0, y3 = 0.0, gx = 0.0, gy = 0.0;
  __device__ inline void add(double vx, double vy, double f, double g) {
    r += f; mx += vx * f; my += vy * f;
    e += 0.5 * (vx * vx + vy * vy) * f + g;
    if (SK) {
      const double v2 = vx * vx + vy * vy;
      xx += vx * vx * f; xy += vx * vy * f; yy += vy * vy * f;
      x3 += vx * v2 * f; y3 += vy * v2 * f;
      gx += vx * g; gy += vy * g;
    }
  }
  template <class Red>
  __device__ inline void reduce(Red red) {
    r = red(r); mx = red(mx); my = red(my); e = red(e);
    if (SK) {
      xx = red(xx); xy = red(xy); yy = red(yy); x3 = red(x3); y3 = red(y3);
      gx = red(gx); gy = red(gy);
    }
  }
  // mo = (rho, ux, uy, T); with SK hq = (qx, qy).  w = dv^2.
  __device__ inline void finish(double w, double* mo, double* hq) const {
    const double rho = r * w, ux = mx * w / rho, uy = my * w / rho, en = e * w;
    mo[0] = rho; mo[1] = ux; mo[2] = uy;
    mo[3] = (2.0 * en / rho - (ux * ux + uy * uy)) / 3.0;
    if (SK) {
      const double sxx = xx * w, sxy = xy * w, syy = yy * w, tr = sxx + syy;
      const double g0 = en - 0.5 * tr, u2 = ux * ux + uy * uy;
      hq[0] = 0.5 * (x3 * w - 2.0 * (sxx * ux + sxy * uy) - ux * tr + 2.0 * rho * u2 * ux) + gx * w - ux * g0;
      hq[1] = 0.5 * (y3 * w - 2.0 * (sxy * ux + syy * uy) - uy * tr + 2.0 * rho * u2 * uy) + gy * w - uy * g0;
    }
  }
};

// Reduced Shakhov equilibria (eq. ShakhovDD) from the Maxwellian value M at
// v, with c = v - u:  f_eq = M [1 + s (|c|^2/T - 4)],
// g_eq = T/2 M [1 + s (|c|^2/T - 2)],  s = (1 - Pr) c.q / (5 P T), P = rho T
// (R = 1).  a = (1 - Pr)/(5 rho T^2), invT = 1/T.
__device__ inline void shakhov2(double a, double qx, double qy, double T, double invT, double cx,
                                double cy, double M, double& Ef, double& Eg) {
  const double s = a * (cx * qx + cy * qy);
  const double c2T = (cx * cx + cy * cy) * invT;
  Ef = M * (1.0 + s * (c2T - 4.0));
  Eg = 0.5 * T * M * (1.0 + s * (c2T - 2.0));
}

// Block-wide sum over the 4 waves of a 256-thread block; every thread gets
// the total.  Waves are added in wave order (deterministic).
__device__ inline double block_sum4(double v, double* lds) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[wave] = v;
  __syncthreads();
  return ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

// Block-wide sums of two values at once (same order as block_sum4).
__device__ inline void block_sum4x2(double& a, double& b, double* lds) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) { lds[wave] = a; lds[4 + wave] = b; }
  __syncthreads();
  a = ((lds[0] + lds[1]) + lds[2]) + lds[3];
  b = ((lds[4] + lds[5]) + lds[6]) + lds[7];
}

// One control volume's members, staged in LDS by the block that updates
// it: the rows read through each member's four edges (the volume's own row
// where an edge is closed; its open length is then 0), the rows it writes,
// and its wall edges with the per-axis factors of their Maxwellians
// (exp(-(v - u_w)^2 / 2T_w) along each axis, so M_w = c_w fx[p1] fy[p2]).
struct CvStage {
  const double2* src[kMaxMembers][4];   // +x, -x, +y, -y
  double len[kMaxMembers][4];
  double2* dst[kMaxMembers];            // nullptr: not written
  int live[kMaxMembers];                // 0: written as zero (cell now solid)
  double wall[kMaxMembers][8];          // L_w, n_w, u_w, r_w - centre, phi_w
  double wfx[kMaxMembers][kMaxN2], wfy[kMaxMembers][kMaxN2];
  double eqx[kMaxN2], eqy[kMaxN2];      // per-axis factors of the volume's Maxwellian
  double red[8];
  int nwall;
};

// ---------------------------------------------------------------------
// The update of one control volume that is cut or owns merged cells, by a
// block of 256 threads (velocities strided over the block).  Wall density
// of each wall edge (eq. BoundaryDDv), fluxes of all members' edges (eq.
// FluxDD), the explicit update with relaxation (eq. ExSchemeDD; ratio and
// dts carry the area change S^n / S^{n+1,*} of a moving body, eq. SchemeDD), the new
// value written to every member (eq. UpdateDD), the wall stress of the
// state at t^n summed into force and torque (eqs. StressTensorDD,
// eq-force, eq-torque) and the velocity sums of the new value.  The
// caller has staged dst and live of each member.
// ---------------------------------------------------------------------
template <bool SK>
__device__ void cv_update(CvStage& cs, const Geo2D& G, const int* __restrict__ mem, int nm,
                          const double2* __restrict__ in, const double2* __restrict__ own,
                          const double* __restrict__ body, const StepParams& P, double rho,
                          double ux, double uy, double T, double qx, double qy, double dtau,
                          double ratio, double dts,
                          Sums2<SK>& sm, double& Fx, double& Fy, double& Tq) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int N = G.N, nvel = G.nvel, nx = G.nx, ny = G.ny;
  const double inv2T = 0.5 / T, A = rho / (2.0 * M_PI * T);
  const double ska = SK ? P.sk_coef / (rho * T * T) : 0.0;
  const double Tw = P.t_wall, cw = 1.0 / (2.0 * M_PI * Tw), inv2Tw = 0.5 / Tw;
  if (tid < kWave) {
    const int t = tid;
    const int k = t < nm ? mem[t] : 0;
    const bool isw = t < nm && G.lw[k] > 0.0;
    const unsigned long long wm = __ballot(isw);
    if (t < nm) {
      const int i = k % nx, j = k / nx;
      const double Lr = G.lxp[k], Ll = G.lxm[k], Lt = G.lyp[k], Lb = G.lym[k];
      cs.src[t][0] = Lr > 0.0 ? (i + 1 < nx ? in + (size_t)(k + 1) * nvel : G.ghost) : own;
      cs.src[t][1] = Ll > 0.0 ? (i > 0 ? in + (size_t)(k - 1) * nvel : G.ghost) : own;
      cs.src[t][2] = Lt > 0.0 ? (j + 1 < ny ? in + (size_t)(k + nx) * nvel : G.ghost) : own;
      cs.src[t][3] = Lb > 0.0 ? (j > 0 ? in + (size_t)(k - nx) * nvel : G.ghost) : own;
      cs.len[t][0] = Lr > 0.0 ? Lr : 0.0;
      cs.len[t][1] = Ll > 0.0 ? Ll : 0.0;
      cs.len[t][2] = Lt > 0.0 ? Lt : 0.0;
      cs.len[t][3] = Lb > 0.0 ? Lb : 0.0;
    }
    if (isw) {
      const int u = __popcll(wm & ((1ull << t) - 1));
      double uwx, uwy;
      const double rx = G.rwx[k], ry = G.rwy[k];
      wall_velocity(body, rx, ry, &uwx, &uwy);
      double* wd = cs.wall[u];
      wd[0] = G.lw[k]; wd[1] = G.nwx[k]; wd[2] = G.nwy[k];
      wd[3] = uwx; wd[4] = uwy; wd[5] = rx - body[0]; wd[6] = ry - body[1];
    }
    if (t == 0) cs.nwall = __popcll(wm);
  }
  __syncthreads();
  const int nwall = cs.nwall;
  for (int a = tid; a < nwall * N; a += nth) {
    const int u = a / N, c = a % N;
    const double v = vnode(P.vmin, P.dv, c);
    const double ex = v - cs.wall[u][3], ey = v - cs.wall[u][4];
    cs.wfx[u][c] = exp(-ex * ex * inv2Tw);
    cs.wfy[u][c] = exp(-ey * ey * inv2Tw);
  }
  if (dtau != 0.0)
    for (int a = tid; a < N; a += nth) {
      const double v = vnode(P.vmin, P.dv, a);
      const double ex = v - ux, ey = v - uy;
      cs.eqx[a] = exp(-ex * ex * inv2T);
      cs.eqy[a] = exp(-ey * ey * inv2T);
    }
  __syncthreads();
  // wall density of each wall edge: no net mass through it (eq. BoundaryDDv)
  for (int u = 0; u < nwall; ++u) {
    const double nwx = cs.wall[u][1], nwy = cs.wall[u][2], uwx = cs.wall[u][3], uwy = cs.wall[u][4];
    double num = 0.0, den = 0.0;
    for (int p = tid; p < nvel; p += nth) {
      const int p1 = p % N, p2 = p / N;
      const double vx = vnode(P.vmin, P.dv, p1), vy = vnode(P.vmin, P.dv, p2);
      const double cn = (vx - uwx) * nwx + (vy - uwy) * nwy;
      const double fo = own[p].x;
      const double Mw = cw * cs.wfx[u][p1] * cs.wfy[u][p2];
      num += cn > 0.0 ? cn * fo : 0.0;
      den += cn < 0.0 ? cn * Mw : 0.0;
    }
    block_sum4x2(num, den, cs.red);
    if (tid == 0) cs.wall[u][7] = den != 0.0 ? -num / den : 0.0;
  }
  __syncthreads();
  double fx = 0.0, fy = 0.0, tq = 0.0;
  for (int p = tid; p < nvel; p += nth) {
    const int p1 = p % N, p2 = p / N;
    const double vx = vnode(P.vmin, P.dv, p1), vy = vnode(P.vmin, P.dv, p2);
    const double vxm = fmin(vx, 0.0), vxp = fmax(vx, 0.0);
    const double vym = fmin(vy, 0.0), vyp = fmax(vy, 0.0);
    const double2 o = own[p];
    double Rf = 0.0, Rg = 0.0;
    for (int t = 0; t < nm; ++t) {
      const double2 nr = cs.src[t][0][p], nl = cs.src[t][1][p];
      const double2 nt = cs.src[t][2][p], nb = cs.src[t][3][p];
      const double wr = cs.len[t][0], wl = cs.len[t][1], wt = cs.len[t][2], wb = cs.len[t][3];
      Rf += wr * (vxm * nr.x + vxp * o.x);
      Rg += wr * (vxm * nr.y + vxp * o.y);
      Rf -= wl * (vxm * o.x + vxp * nl.x);
      Rg -= wl * (vxm * o.y + vxp * nl.y);
      Rf += wt * (vym * nt.x + vyp * o.x);
      Rg += wt * (vym * nt.y + vyp * o.y);
      Rf -= wb * (vym * o.x + vyp * nb.x);
      Rg -= wb * (vym * o.y + vyp * nb.y);
    }
    for (int u = 0; u < nwall; ++u) {
      const double* wd = cs.wall[u];
      const double Lw = wd[0];
      const double cx_ = vx - wd[3], cy_ = vy - wd[4];
      const double cn = cx_ * wd[1] + cy_ * wd[2];
      const double Mw = cw * cs.wfx[u][p1] * cs.wfy[u][p2];
      const double fw = wd[7] * Mw, gw = wd[7] * 0.5 * Tw * Mw;
      Rf += Lw * (fmin(cn, 0.0) * fw + fmax(cn, 0.0) * o.x);
      Rg += Lw * (fmin(cn, 0.0) * gw + fmax(cn, 0.0) * o.y);
      const double fv = cn < 0.0 ? fw : (cn > 0.0 ? o.x : 0.0);
      const double sw = Lw * cn * fv;
      fx += cx_ * sw;
      fy += cy_ * sw;
      tq += (wd[5] * cy_ - wd[6] * cx_) * sw;
    }
    double E = 0.0, Eg = 0.0;
    if (dtau != 0.0) {
      E = A * cs.eqx[p1] * cs.eqy[p2];
      if (SK) shakhov2(ska, qx, qy, T, 1.0 / T, vx - ux, vy - uy, E, E, Eg);
      else Eg = 0.5 * T * E;
    }
    const double fn = ratio * o.x - dts * Rf + ratio * dtau * (E - o.x);
    const double gn = ratio * o.y - dts * Rg + ratio * dtau * (Eg - o.y);
    for (int t = 0; t < nm; ++t) {
      double2* d = cs.dst[t];
      if (d) d[p] = cs.live[t] ? make_double2(fn, gn) : make_double2(0.0, 0.0);
    }
    sm.add(vx, vy, fn, gn);
  }
  Fx = block_sum4(fx, cs.red) * P.w;
  Fy = block_sum4(fy, cs.red) * P.w;
  Tq = block_sum4(tq, cs.red) * P.w;
  sm.reduce([&](double v) { return block_sum4(v, cs.red); });
}

// A cut or merged control volume of a fixed geometry.  With write_state ==
// 0 only the force is produced.
template <bool SK>
__device__ void cut_cv(const Geo2D& G, const double2* __restrict__ in, double2* __restrict__ out,
                       double* __restrict__ mom, double* __restrict__ heat, double* __restrict__ fslot,
                       double* __restrict__ mpart, const double* __restrict__ body,
                       const StepParams& P, int q, CvStage& cs) {
  const int tid = threadIdx.x;
  const int m = G.irr[q];
  const int b = G.mptr[q];
  // more members than supported is reported by the list builder; never index past the arrays
  const int nm = min(G.mptr[q + 1] - b, kMaxMembers);
  const int nvel = G.nvel;
  const double rho = mom[4 * m + 0], ux = mom[4 * m + 1], uy = mom[4 * m + 2], T = mom[4 * m + 3];
  const double dtau = P.tau_coef > 0.0 && !P.implicit ? P.dt * rho / P.tau_coef : 0.0;
  const double qx = SK ? heat[2 * m] : 0.0, qy = SK ? heat[2 * m + 1] : 0.0;
  const double S = G.scv[m];
  if (tid < nm) {
    cs.dst[tid] = P.write_state ? out + (size_t)G.mem[b + tid] * nvel : nullptr;
    cs.live[tid] = 1;
  }
  Sums2<SK> sm;
  double Fx, Fy, Tq;
  cv_update<SK>(cs, G, G.mem + b, nm, in, in + (size_t)m * nvel, body, P, rho, ux, uy, T, qx, qy,
                dtau, 1.0, P.dt / S, sm, Fx, Fy, Tq);
  if (tid == 0) {
    double mo[4], hq[2];
    sm.finish(P.w, mo, hq);
    if (P.write_state)
      for (int t = 0; t < nm; ++t) {
        const int k = G.mem[b + t];
        for (int i = 0; i < 4; ++i) mom[4 * k + i] = mo[i];
        if (SK) { heat[2 * k] = hq[0]; heat[2 * k + 1] = hq[1]; }
      }
    fslot[3 * q + 0] = Fx;
    fslot[3 * q + 1] = Fy;
    fslot[3 * q + 2] = Tq;
    if (mpart) *mpart = S * mo[0];
  }
}

__global__ void __launch_bounds__(256) k_cut_force2d(Geo2D G, const double2* __restrict__ in,
                                                     double* __restrict__ mom,
                                                     double* __restrict__ fslot,
                                                     const double* __restrict__ body,
                                                     StepParams P) {
  __shared__ CvStage cs;
  for (int q = blockIdx.x; q < G.counts[0]; q += gridDim.x)
    cut_cv<false>(G, in, nullptr, mom, nullptr, fslot, nullptr, body, P, q, cs);
}

// ---------------------------------------------------------------------
// The fused step: one launch per time step.
// Two launches per time step.  k_cutstep2d: one 256-thread block per cut /
// merged control volume (kept apart so that its per-member bookkeeping does
// not set the register budget of the streaming kernel).  k_step2d:
//   block 0           deferred deterministic reduction of the previous
//                     step's force slots and mass partials into diag
//   blocks 8..        regular-cell tiles: kTileW adjacent columns x a
//                     segment of rows, one wave per column marching up
//                     the rows.  The wave keeps in registers the upper
//                     velocity half (v_y > 0) of the cell below and the
//                     lower half (v_y < 0) of the current cell, so every
//                     value of the state is loaded from HBM once; the x
//                     upwind neighbour comes from the adjacent wave's loads
//                     through L2.  Tiles are mapped so that the tiles of
//                     one XCD are adjacent columns of the same rows.
// ---------------------------------------------------------------------
constexpr int kTileW = 4;   // columns (waves) per tile
constexpr int kListBlocks = 512;   // grid of kernels that walk a list whose length is on the device
constexpr int kPrefetch = 4;       // chunks loaded ahead of the one computed, at most
// VGPRs the Shakhov variant needs beyond the BGK one (heat-flux sums, q and
// the velocity offsets), taken from the prefetch budget
constexpr int kSkRegs = 40;
// VGPRs per chunk the semi-implicit variant needs beyond the explicit one
// (it holds the transported row until its relaxation)
constexpr int kImRegs = 8;
// Chunks loaded ahead of the one computed.  Each chunk in flight costs 16
// VGPRs and the row window 8 per chunk; the depth is capped so that a wave
// stays within 256 VGPRs (2 waves per SIMD) without spilling.
constexpr int prefetch_depth(int nch, bool sk = false, bool im = false) {
  int cap = (138 - (sk ? kSkRegs : 0) - (im ? kImRegs * nch : 0) - 8 * nch) / 16;
  int d = kPrefetch < cap ? kPrefetch : cap;
  d = d < 1 ? 1 : d;
  return d < nch - 1 ? d : (nch - 1 > 0 ? nch - 1 : 0);
}

struct FusedArgs {
  const int* kind;          // per-cell dispatch kind (KIND_REGULAR cells are streamed)
  const double2* in;
  double2* out;
  double* mom;
  double* heat;             // Shakhov: heat flux (qx, qy) per cell, else unused
  double* fslot;            // this step: 3 per control volume
  double* mpart;            // this step: ntiles tile partials, then n_irr
  const double* prev_fslot; // previous step (deferred reduction), may be null
  const double* prev_mpart;
  double* red_force;        // diag row of the previous step (force, torque)
  double* red_mass;         // diag mass of the state entering this step
  const double* body;
  int n_cut, cut_base;      // cut blocks start at block cut_base
  int ntiles, tile_base, ntiles_pad;
  int ngroups, seglen;
  int split;                // number of velocity rows with v_y < 0
};

__device__ void deferred_reduce(const Geo2D& G, const FusedArgs& A, double* lds) {
  const int nparts = A.ntiles + A.n_cut;
  double ms = 0.0, fx = 0.0, fy = 0.0, tq = 0.0;
  for (int t = threadIdx.x; t < nparts; t += blockDim.x) ms += A.prev_mpart[t];
  for (int q = threadIdx.x; q < A.n_cut; q += blockDim.x) {
    fx += A.prev_fslot[3 * q]; fy += A.prev_fslot[3 * q + 1]; tq += A.prev_fslot[3 * q + 2];
  }
  ms = block_sum4(ms, lds); fx = block_sum4(fx, lds);
  fy = block_sum4(fy, lds); tq = block_sum4(tq, lds);
  if (threadIdx.x == 0) {
    if (A.red_force) { A.red_force[0] = fx; A.red_force[1] = fy; A.red_force[2] = tq; }
    if (A.red_mass) A.red_mass[0] = ms;
  }
}

typedef double d2v __attribute__((ext_vector_type(2)));
// a type in the global address space: pointers read from memory (the
// batched kernels' descriptor tables) carry no address space, and the
// compiler then issues flat operations, which count on both the vector
// memory and the LDS counters, so that every wait drains both
template <class T>
using glob = __attribute__((address_space(1))) T;

// load one velocity half of a cell row (or of the farfield table)
template <int NCH>
__device__ inline void load_half(d2v (&dst)[NCH], const glob<d2v>* __restrict__ row, int base,
                                 int count, int lane) {
#pragma unroll
  for (int k = 0; k < NCH; ++k) {
    const int o = k * 64 + lane;
    dst[k] = o < count ? row[base + o] : d2v{0.0, 0.0};
  }
}

// One tile of regular cells.  Velocity rows [0, split) have v_y < 0 (lower
// half, y-upwind neighbour above), rows [split, N) have v_y >= 0 (upper
// half, y-upwind neighbour below).  Both halves are walked together, chunk
// by chunk: chunk k of either half holds the same p1 for a given lane, so
// the x-upwind cell and the x part of the Maxwellian are shared.
// Everything the regular-cell tile needs, passed by value so that it lives
// in scalar registers.
struct TileArgs {
  const int* kind;
  const double2* in;
  double2* out;
  double* mom;
  double* heat;
  double* mpart;
  const double2* ghost;
  int nx, ny, N, nvel, ngroups, seglen, split;
  double dx, dy;
};

__host__ __device__ inline TileArgs tile_args(const Geo2D& G, const FusedArgs& A) {
  TileArgs T;
  T.kind = A.kind; T.in = A.in; T.out = A.out; T.mom = A.mom; T.heat = A.heat; T.mpart = A.mpart;
  T.ghost = G.ghost;
  T.nx = G.nx; T.ny = G.ny; T.N = G.N; T.nvel = G.nvel;
  T.ngroups = A.ngroups; T.seglen = A.seglen; T.split = A.split;
  T.dx = G.dx; T.dy = G.dy;
  return T;
}

// xlo (nullable): LDS of kTileW x NCH x 64 values.  At each row every wave
// publishes the lower half of its cell there, and the waves of the tile read
// their x-upwind lower halves from it: that half was loaded by its owner one
// row earlier (as the y-upwind of the row below), so its lines have left L2
// by the time the neighbours need them.  (The upper half is loaded by its
// owner in the same row and comes through L2.)
// IM: semi-implicit step (ImpSchemeDD, direct equilibrium).  The row's
// transported value is written as usual, its moments give the equilibrium,
// and the wave then reads the value back (its lines are still in L2),
// relaxes it implicitly with dt/tau of the state entering the step, writes
// it and sums the moments of the result.
template <int NCH, bool SK, bool IM = false>
__device__ void regular_tile(const TileArgs Ta, const StepParams P, int tile, double* lds,
                             d2v* xlo = nullptr) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int gi = tile % Ta.ngroups, seg = tile / Ta.ngroups;
  const int i = gi * kTileW + wave;
  const int nx = Ta.nx, ny = Ta.ny, N = Ta.N, nvel = Ta.nvel;
  const int j0 = seg * Ta.seglen, j1 = min(j0 + Ta.seglen, ny);
  const int split = Ta.split;
  const int lo_n = split * N, hi_n = nvel - lo_n;   // sizes of the two halves
  const glob<d2v>* in = (const glob<d2v>*)Ta.in;
  glob<d2v>* out = (glob<d2v>*)Ta.out;
  const glob<d2v>* ghost = (const glob<d2v>*)Ta.ghost;
  const glob<int>* kind = (const glob<int>*)Ta.kind;
  glob<double>* mom = (glob<double>*)Ta.mom;
  glob<double>* heat = (glob<double>*)Ta.heat;
  double msum = 0.0;
  if (i < nx && j0 < j1) {
    const double S = Ta.dx * Ta.dy;
    const double cxf = P.dt / S * Ta.dy, cyf = P.dt / S * Ta.dx;
    // IM: the lower halves live only in LDS, in two buffers (this row's,
    // read by the wave and its x-neighbours; the next row's, written as it
    // is loaded), which frees the registers for the transported row
    d2v prevU[NCH], curL[IM ? 1 : NCH];
    load_half<NCH>(prevU, j0 > 0 ? in + (size_t)((j0 - 1) * nx + i) * nvel : ghost, lo_n, hi_n, lane);
    if constexpr (IM) {
      const glob<d2v>* r0 = in + (size_t)(j0 * nx + i) * nvel;
#pragma unroll
      for (int k = 0; k < NCH; ++k)
        xlo[(wave * NCH + k) * kWave + lane] = k * 64 + lane < lo_n ? r0[k * 64 + lane] : d2v{0.0, 0.0};
    } else {
      load_half<NCH>(curL, in + (size_t)(j0 * nx + i) * nvel, 0, lo_n, lane);
    }
    for (int j = j0; j < j1; ++j) {
      d2v* xcur = xlo;
      d2v* xnext = xlo;
      if constexpr (IM) {
        __syncthreads();   // row j's lower halves are complete, row j-1's are no longer read
        const int par = (j - j0) & 1;
        xcur = xlo + par * (kTileW * NCH * kWave);
        xnext = xlo + (1 - par) * (kTileW * NCH * kWave);
      } else if (xlo) {
        __syncthreads();   // every wave is done with the previous row's halves
#pragma unroll
        for (int k = 0; k < NCH; ++k) xlo[(wave * NCH + k) * kWave + lane] = curL[k];
        __syncthreads();
      }
      const int c = j * nx + i;
      const glob<d2v>* row = in + (size_t)c * nvel;
      const glob<d2v>* nrow = j + 1 < ny ? row + (size_t)nx * nvel : ghost;
      const bool reg = kind[c] == KIND_REGULAR;   // uniform over the wave
      double Am = 0.0, T = 1.0, dtau = 0.0, tx = 0.0, ty = 0.0, nu = 0.0;
      double ux = 0.0, uy = 0.0, qx = 0.0, qy = 0.0, ska = 0.0, invT = 1.0;   // SK only
      if (reg) {
        const glob<double>* mc = mom + 4 * c;
        const double rho = mc[0];
        ux = mc[1]; uy = mc[2];
        T = mc[3];
        const double inv2T = 0.5 / T;
        Am = rho / (2.0 * M_PI * T);
        dtau = P.tau_coef > 0.0 && !IM ? P.dt * rho / P.tau_coef : 0.0;
        nu = IM && P.tau_coef > 0.0 ? P.dt * rho / P.tau_coef : 0.0;
        if (SK) {
          qx = heat[2 * c]; qy = heat[2 * c + 1];
          ska = P.sk_coef / (rho * T * T);
          invT = 1.0 / T;
        }
        if (!IM && lane < N) {
          const double v = vnode(P.vmin, P.dv, lane);
          tx = exp(-(v - ux) * (v - ux) * inv2T);
          ty = exp(-(v - uy) * (v - uy) * inv2T);
        }
      }
      const glob<d2v>* xl = i > 0 ? row - nvel : ghost;        // x-upwind for v_x > 0
      const glob<d2v>* xr = i + 1 < nx ? row + nvel : ghost;   // x-upwind for v_x < 0
      glob<d2v>* orow = out + (size_t)c * nvel;
      Sums2<SK> sm;
      // software pipeline over the chunks: the loads of chunk k+PD are issued
      // before chunk k is computed; a scheduling barrier between chunks keeps
      // the live set to the window plus PD+1 chunks.
      // The per-chunk velocity constants are the same for every row; they are
      // recomputed per row (a few ALU ops) instead of being held in registers
      // across the row loop, which would cost ~10 VGPRs per chunk.
      int lv = lane;
      asm volatile("" : "+v"(lv));
      constexpr int PD = prefetch_depth(NCH, SK, IM);
      d2v bN[NCH], bU[NCH], bXa[NCH], bXb[NCH];
      d2v fsL[IM ? NCH : 1], fsU[IM ? NCH : 1];   // IM: the transported row
      // lanes whose x-upwind cell is another wave of this tile read its
      // lower half from xlo (v_x > 0: the wave to the left)
      auto xwave = [&](int k) {
        const bool pos = vnode(P.vmin, P.dv, (k * 64 + lv) % N) > 0.0;
        const bool in_tile = pos ? wave > 0 : (wave + 1 < kTileW && i + 1 < nx);
        return xlo && in_tile ? (pos ? wave - 1 : wave + 1) : -1;
      };
      // Every lane issues the same loads for every chunk and row (lanes past
      // a half read its first element, lanes whose x-upwind lower half comes
      // from xlo read the x-upwind upper half, which the bXb load brings
      // in), so the loads carry no branch: the compiler then waits for each
      // chunk's loads alone instead of draining the whole prefetch window.
      // Values of such lanes are never used.
      auto issue = [&](int k) {
        const int o = k * 64 + lv;
        const int lp1 = o % N;
        const glob<d2v>* xrow = vnode(P.vmin, P.dv, lp1) > 0.0 ? xl : xr;
        const int oa = o < lo_n ? o : 0, ob = o < hi_n ? o : 0;
        bN[k] = nrow[oa];
        bU[k] = row[lo_n + ob];
        bXa[k] = xrow[xwave(k) < 0 ? oa : lo_n + ob];
        bXb[k] = xrow[lo_n + ob];
      };
#pragma unroll
      for (int k = 0; k < PD; ++k) issue(k);
#pragma unroll
      for (int k = 0; k < NCH; ++k) {
        if (k + PD < NCH) issue(k + PD);
        const int o = k * 64 + lv;
        const int xw = xwave(k);
        const d2v nL = bN[k], cU = bU[k], xb = bXb[k];
        // the LDS value is read by every lane (from its own slot where it is
        // not used) and selected as a value: a select of the two sources'
        // addresses would put bXa in scratch and read both through flat loads
        const d2v xs = xlo ? xcur[((xw >= 0 ? xw : wave) * NCH + k) * kWave + lv] : d2v{0.0, 0.0};
        const d2v xa = xw >= 0 && o < lo_n ? xs : bXa[k];
        if (reg) {
          const int p1 = o % N, q2 = o / N;
          const double vx = vnode(P.vmin, P.dv, p1);
          const double ax = cxf * fabs(vx);
          const double ex = Am * __shfl(tx, p1, 64);
          const double tyl = __shfl(ty, q2 < N ? q2 : 0, 64);
          const double tyu = __shfl(ty, split + q2 < N ? split + q2 : 0, 64);
          {   // lower half: v_y < 0, y-upwind is the cell above
            const bool va = o < lo_n;
            const double vy = vnode(P.vmin, P.dv, q2);
            const double ay = cyf * fabs(vy);
            d2v own;
            if constexpr (IM) own = xcur[(wave * NCH + k) * kWave + lv];
            else own = curL[k];
            double fn = own.x - ax * (own.x - xa.x) - ay * (own.x - nL.x);
            double gn = own.y - ax * (own.y - xa.y) - ay * (own.y - nL.y);
            if (!IM) {
              double E = ex * tyl, Eg = 0.5 * T * E;
              if (SK) shakhov2(ska, qx, qy, T, invT, vx - ux, vy - uy, ex * tyl, E, Eg);
              fn += dtau * (E - own.x);
              gn += dtau * (Eg - own.y);
            }
            if (IM) fsL[k] = d2v{fn, gn};
            else if (va) __builtin_nontemporal_store(d2v{fn, gn}, &orow[o]);
            sm.add(vx, vy, va ? fn : 0.0, va ? gn : 0.0);
          }
          {   // upper half: v_y >= 0, y-upwind is the cell below
            const bool vb = o < hi_n;
            const double vy = vnode(P.vmin, P.dv, split + q2);
            const double ay = cyf * fabs(vy);
            const d2v own = cU, yu = prevU[k];
            double fn = own.x - ax * (own.x - xb.x) - ay * (own.x - yu.x);
            double gn = own.y - ax * (own.y - xb.y) - ay * (own.y - yu.y);
            if (!IM) {
              double E = ex * tyu, Eg = 0.5 * T * E;
              if (SK) shakhov2(ska, qx, qy, T, invT, vx - ux, vy - uy, ex * tyu, E, Eg);
              fn += dtau * (E - own.x);
              gn += dtau * (Eg - own.y);
            }
            if (IM) fsU[k] = d2v{fn, gn};
            else if (vb) __builtin_nontemporal_store(d2v{fn, gn}, &orow[lo_n + o]);
            sm.add(vx, vy, vb ? fn : 0.0, vb ? gn : 0.0);
          }
        }
        prevU[k] = cU;
        if constexpr (IM) xnext[(wave * NCH + k) * kWave + lv] = nL;
        else curL[k] = nL;
        __builtin_amdgcn_sched_barrier(0);
      }
      if (reg && IM) {
        // implicit relaxation toward the equilibrium of the transported row
        sm.reduce([](double v) { return wave_sum(v); });
        double m1[4], h1[2];
        sm.finish(P.w, m1, h1);          // every lane: the sums are wave totals
        const double T1 = m1[3], i2T1 = 0.5 / T1, A1 = m1[0] / (2.0 * M_PI * T1);
        const double sk1 = SK ? P.sk_coef / (m1[0] * T1 * T1) : 0.0, iT1 = 1.0 / T1;
        const double sc = 1.0 / (1.0 + nu);
        double t1x = 0.0, t1y = 0.0;
        if (lane < N) {
          const double v = vnode(P.vmin, P.dv, lane);
          t1x = exp(-(v - m1[1]) * (v - m1[1]) * i2T1);
          t1y = exp(-(v - m1[2]) * (v - m1[2]) * i2T1);
        }
        Sums2<SK> s2;
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
          const int o = k * 64 + lv;
          const int p1 = o % N, q2 = o / N;
          const double vx = vnode(P.vmin, P.dv, p1);
          const double ex = A1 * __shfl(t1x, p1, 64);
          const double tyl = __shfl(t1y, q2 < N ? q2 : 0, 64);
          const double tyu = __shfl(t1y, split + q2 < N ? split + q2 : 0, 64);
          if (o < lo_n) {
            const double vy = vnode(P.vmin, P.dv, q2);
            double E = ex * tyl, Eg = 0.5 * T1 * E;
            if (SK) shakhov2(sk1, h1[0], h1[1], T1, iT1, vx - m1[1], vy - m1[2], ex * tyl, E, Eg);
            const d2v fs = fsL[k];
            const double fn = (fs.x + nu * E) * sc, gn = (fs.y + nu * Eg) * sc;
            __builtin_nontemporal_store(d2v{fn, gn}, &orow[o]);
            s2.add(vx, vy, fn, gn);
          }
          if (o < hi_n) {
            const double vy = vnode(P.vmin, P.dv, split + q2);
            double E = ex * tyu, Eg = 0.5 * T1 * E;
            if (SK) shakhov2(sk1, h1[0], h1[1], T1, iT1, vx - m1[1], vy - m1[2], ex * tyu, E, Eg);
            const d2v fs = fsU[k];
            const double fn = (fs.x + nu * E) * sc, gn = (fs.y + nu * Eg) * sc;
            __builtin_nontemporal_store(d2v{fn, gn}, &orow[lo_n + o]);
            s2.add(vx, vy, fn, gn);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        s2.reduce([](double v) { return wave_sum(v); });
        if (lane == 0) {
          double mo[4], hq[2];
          s2.finish(P.w, mo, hq);
          glob<double>* dst = mom + 4 * c;
          dst[0] = mo[0]; dst[1] = mo[1]; dst[2] = mo[2]; dst[3] = mo[3];
          if (SK) { heat[2 * c] = hq[0]; heat[2 * c + 1] = hq[1]; }
        }
        msum += S * (s2.r * P.w);
      } else if (reg) {
        sm.reduce([](double v) { return wave_sum(v); });
        if (lane == 0) {
          double mo[4], hq[2];
          sm.finish(P.w, mo, hq);
          glob<double>* dst = mom + 4 * c;
          dst[0] = mo[0]; dst[1] = mo[1]; dst[2] = mo[2]; dst[3] = mo[3];
          if (SK) { heat[2 * c] = hq[0]; heat[2 * c + 1] = hq[1]; }
        }
        msum += S * (sm.r * P.w);
      }
    }
  }
  if (xlo && !(i < nx) && j0 < j1)   // columns past the grid still take part in the row barriers
    for (int j = j0; j < j1; ++j) {
      __syncthreads();
      if (!IM) __syncthreads();
    }
  __syncthreads();
  if (lane == 0) lds[wave] = msum;
  __syncthreads();
  if (threadIdx.x == 0) ((glob<double>*)Ta.mpart)[tile] = ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

// regular-cell tiles (+ block 0: deferred reduction of the previous step)
template <int NCH, bool SK, bool IM>
__device__ __forceinline__ void step_tiles(const Geo2D& G, const FusedArgs& A, const StepParams& P) {
  __shared__ double lds[8];
  // LDS lower halves (<= 64 KB per block); the semi-implicit variant keeps
  // two rows of them and needs them
  constexpr bool kX = NCH <= 16;
  static_assert(!IM || NCH <= 8, "semi-implicit tile: at most 8 chunks per half");
  __shared__ d2v xlo[kX ? (IM ? 2 : 1) * kTileW * NCH * kWave : 1];
  const int bid = blockIdx.x;
  if (bid < A.tile_base) {
    if (bid == 0 && A.prev_mpart) deferred_reduce(G, A, lds);
    return;
  }
  // XCD-aware order: block b runs on XCD b % 8; the tiles of one XCD are
  // contiguous in the tile order (adjacent columns, same rows)
  const int b = bid - A.tile_base;
  const int per = A.ntiles_pad / 8;
  const int tile = (b % 8) * per + b / 8;
  if (tile >= A.ntiles) return;
  regular_tile<NCH, SK, IM>(tile_args(G, A), P, tile, lds, kX ? xlo : nullptr);
}

template <int NCH, bool SK>
__global__ void __launch_bounds__(256) k_step2d(Geo2D G, FusedArgs A, StepParams P) {
  step_tiles<NCH, SK, false>(G, A, P);
}

// the semi-implicit variant is held to 2 waves per SIMD (its LDS allows 2
// blocks per CU); a few spilled registers cost less than half the waves
template <int NCH, bool SK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_step2d_im(Geo2D G, FusedArgs A, StepParams P) {
  step_tiles<NCH, SK, true>(G, A, P);
}

// cut / merged control volumes of one step, one 256-thread block each
__global__ void __launch_bounds__(256) k_cutstep2d(Geo2D G, FusedArgs A, StepParams P) {
  __shared__ CvStage cs;
  const int q = blockIdx.x;
  if (P.shakhov)
    cut_cv<true>(G, A.in, A.out, A.mom, A.heat, A.fslot, A.mpart + A.ntiles + q, A.body, P, q, cs);
  else
    cut_cv<false>(G, A.in, A.out, A.mom, nullptr, A.fslot, A.mpart + A.ntiles + q, A.body, P, q, cs);
}

// final reduction of the last step of a call (same code as the deferred one)
__global__ void __launch_bounds__(256) k_final_reduce2d(Geo2D G, FusedArgs A) {
  __shared__ double lds[8];
  deferred_reduce(G, A, lds);
}

// ---------------------------------------------------------------------
// Merge (eq. FusionDD) of control volumes with several members, in place,
// followed by the moments of the merged value.  One 256-thread block per
// control volume; its members and their areas are read once, and the
// members' values of a velocity are requested together.
// ---------------------------------------------------------------------
template <bool SK>
__device__ void merge_cv(const Geo2D& G, double2* __restrict__ st, double* __restrict__ mom,
                         double* __restrict__ heat, const StepParams& P, int q, double* lds) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int m = G.irr[q];
  const int b = G.mptr[q], nm = min(G.mptr[q + 1] - b, kMaxMembers);
  const int N = G.N, nvel = G.nvel;
  const double S = G.scv[m];
  int mk[kMaxMembers];
  double w[kMaxMembers];
#pragma unroll
  for (int t = 0; t < kMaxMembers; ++t) {
    mk[t] = t < nm ? G.mem[b + t] : m;
    w[t] = t < nm ? G.sbar[mk[t]] : 0.0;
  }
  Sums2<SK> sm;
  for (int p = tid; p < nvel; p += nth) {
    double af = 0.0, ag = 0.0;
    if (nm > 1) {
      double2 v[kMaxMembers];
      // every member slot is loaded (past the members the master's row,
      // with weight 0), so that no branch splits the loads
#pragma unroll
      for (int t = 0; t < kMaxMembers; ++t) v[t] = st[(size_t)mk[t] * nvel + p];
#pragma unroll
      for (int t = 0; t < kMaxMembers; ++t) { af += w[t] * v[t].x; ag += w[t] * v[t].y; }
      af /= S; ag /= S;
#pragma unroll
      for (int t = 0; t < kMaxMembers; ++t)
        if (t < nm) st[(size_t)mk[t] * nvel + p] = make_double2(af, ag);
    } else {
      const double2 v = st[(size_t)m * nvel + p];
      af = v.x; ag = v.y;
    }
    const double vx = vnode(P.vmin, P.dv, p % N), vy = vnode(P.vmin, P.dv, p / N);
    sm.add(vx, vy, af, ag);
  }
  sm.reduce([&](double v) { return block_sum4(v, lds); });
  if (tid == 0) {
    double mo[4], hq[2];
    sm.finish(P.w, mo, hq);
    for (int t = 0; t < nm; ++t) {
      const int k = mk[t];
      for (int i = 0; i < 4; ++i) mom[4 * k + i] = mo[i];
      if (SK) { heat[2 * k] = hq[0]; heat[2 * k + 1] = hq[1]; }
    }
  }
}

__global__ void __launch_bounds__(256) k_merge2d(Geo2D G, double2* __restrict__ st,
                                                 double* __restrict__ mom, double* __restrict__ heat,
                                                 StepParams P) {
  __shared__ double lds[8];
  for (int q = blockIdx.x; q < G.counts[0]; q += gridDim.x) {
    if (P.shakhov) merge_cv<true>(G, st, mom, heat, P, q, lds);
    else merge_cv<false>(G, st, mom, nullptr, P, q, lds);
  }
}

// moments (rho, u, T; with SK the heat flux) of every non-solid cell, one
// wave per cell
template <bool SK>
__device__ void cell_moments2d(const Geo2D& G, const double2* __restrict__ st, double* __restrict__ mom,
                               double* __restrict__ heat, const StepParams& P, int c, int lane) {
  const int N = G.N, nvel = G.nvel;
  Sums2<SK> sm;
  for (int p = lane; p < nvel; p += kWave) {
    const double2 v = st[(size_t)c * nvel + p];
    sm.add(vnode(P.vmin, P.dv, p % N), vnode(P.vmin, P.dv, p / N), v.x, v.y);
  }
  sm.reduce([](double v) { return wave_sum(v); });
  if (lane == 0) {
    double mo[4], hq[2];
    sm.finish(P.w, mo, hq);
    for (int i = 0; i < 4; ++i) mom[4 * c + i] = mo[i];
    if (SK) { heat[2 * c] = hq[0]; heat[2 * c + 1] = hq[1]; }
  }
}

// regular_only: the cells streamed by the regular-cell kernel only (the cut
// and merged control volumes keep the moments their own kernels stored)
__global__ void __launch_bounds__(256) k_mom2d(Geo2D G, const double2* __restrict__ st,
                                               double* __restrict__ mom, double* __restrict__ heat,
                                               StepParams P, int regular_only) {
  const int lane = threadIdx.x & (kWave - 1);
  const int c = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (c >= G.ncell || G.kind[c] == KIND_SOLID) return;
  if (regular_only && G.kind[c] != KIND_REGULAR) return;
  if (P.shakhov) cell_moments2d<true>(G, st, mom, heat, P, c, lane);
  else cell_moments2d<false>(G, st, mom, nullptr, P, c, lane);
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

// Conservative equilibrium (Section 3.1) of every control volume of the
// current state: replaces the direct moments (rho, u, T) held for the next
// relaxation by the Newton solution; one thread per cell.
__global__ void __launch_bounds__(256) k_newton2d(Geo2D G, double* __restrict__ mom, double vmin,
                                                 double dv) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.ncell) return;
  const int kd = G.kind[c];
  if (kd != KIND_REGULAR && kd != KIND_IRREGULAR) return;
  double* m = mom + 4 * (size_t)c;
  const double rho = m[0], ux = m[1], uy = m[2], T = m[3];
  const double target[4] = {rho, rho * ux, rho * uy, 0.5 * rho * (3.0 * T + ux * ux + uy * uy)};
  double x[4] = {rho, ux, uy, T};
  if (conservative_triplet_2d(x, target, vmin, dv, G.N)) {
    m[0] = x[0]; m[1] = x[1]; m[2] = x[2]; m[3] = x[3];
  }
}

// Semi-implicit step (ImpSchemeDD), first part: dt/tau^n of every control
// volume from the directly computed density of the state at t^n.
__global__ void __launch_bounds__(256) k_imex_nu2d(Geo2D G, const double* __restrict__ mom,
                                                  double* __restrict__ nu, double dt, double tau_coef) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.ncell) return;
  const int kd = G.kind[c];
  if (kd != KIND_REGULAR && kd != KIND_IRREGULAR) return;
  nu[c] = tau_coef > 0.0 ? dt * mom[4 * (size_t)c] / tau_coef : 0.0;
}

// Semi-implicit step, last part: the implicit relaxation of every non-solid
// cell's transported value (f*, g*) toward the equilibrium of its control
// volume's transported moments (direct or conservative triplet in mom):
// f = (f* + nu f_eq)/(1 + nu), g = (g* + nu g_eq)/(1 + nu) (eq. BGKDD or
// ShakhovDD).  Masters also write the direct moments (and the heat flux) of
// the new value to mom_next (heat_next).  One wave per cell.
template <bool SK>
__device__ void relax_cell2d(const Geo2D& G, double2* __restrict__ st, const double* __restrict__ mom,
                             const double* __restrict__ heat, const double* __restrict__ nu,
                             double* __restrict__ mom_next, double* __restrict__ heat_next,
                             const StepParams& P, int c, int m, int lane) {
  const int N = G.N, nvel = G.nvel;
  const double* mc = mom + 4 * (size_t)m;
  const double rho = mc[0], ux = mc[1], uy = mc[2], T = mc[3];
  const double A = rho / (2.0 * M_PI * T), inv2T = 0.5 / T;
  const double qx = SK ? heat[2 * m] : 0.0, qy = SK ? heat[2 * m + 1] : 0.0;
  const double ska = SK ? P.sk_coef / (rho * T * T) : 0.0, invT = 1.0 / T;
  const double nv = nu[m], sc = 1.0 / (1.0 + nv);
  double2* row = st + (size_t)c * nvel;
  Sums2<SK> sm;
  for (int p = lane; p < nvel; p += kWave) {
    const double vx = vnode(P.vmin, P.dv, p % N), vy = vnode(P.vmin, P.dv, p / N);
    const double cx = vx - ux, cy = vy - uy;
    double E = A * exp(-(cx * cx + cy * cy) * inv2T), Eg = 0.5 * T * E;
    if (SK) shakhov2(ska, qx, qy, T, invT, cx, cy, E, E, Eg);
    const double2 o = row[p];
    const double fn = (o.x + nv * E) * sc;
    const double gn = (o.y + nv * Eg) * sc;
    row[p] = make_double2(fn, gn);
    sm.add(vx, vy, fn, gn);
  }
  if (c != m) return;
  sm.reduce([](double v) { return wave_sum(v); });
  if (lane == 0) {
    double hq[2];
    sm.finish(P.w, mom_next + 4 * (size_t)c, hq);
    if (SK) { heat_next[2 * c] = hq[0]; heat_next[2 * c + 1] = hq[1]; }
  }
}

__global__ void __launch_bounds__(256) k_relax2d(Geo2D G, double2* __restrict__ st,
                                                const double* __restrict__ mom,
                                                const double* __restrict__ heat,
                                                const double* __restrict__ nu,
                                                double* __restrict__ mom_next,
                                                double* __restrict__ heat_next, StepParams P) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= G.ncell) return;
  const int m = G.master[c];
  if (m < 0) return;
  if (P.shakhov) relax_cell2d<true>(G, st, mom, heat, nu, mom_next, heat_next, P, c, m, lane);
  else relax_cell2d<false>(G, st, mom, nullptr, nu, mom_next, nullptr, P, c, m, lane);
}

// Semi-implicit step, last part for cut and merged control volumes when the
// regular cells are relaxed inside the streaming kernel: the transported
// value (the same for every member) is relaxed toward the equilibrium of the
// control volume's transported moments and written to every member, whose
// moments (and heat flux) are then replaced in place by those of the new
// value.  One 256-thread block per control volume.
template <bool SK>
__global__ void __launch_bounds__(256) k_relax_cut2d(Geo2D G, double2* __restrict__ st,
                                                    double* __restrict__ mom,
                                                    double* __restrict__ heat,
                                                    const double* __restrict__ nu,
                                                    double* __restrict__ mpart, StepParams P) {
  __shared__ double lds[8];
  const int q = blockIdx.x;
  const int m = G.irr[q];
  const int b = G.mptr[q], e = G.mptr[q + 1];
  const int N = G.N, nvel = G.nvel;
  const double rho = mom[4 * m], ux = mom[4 * m + 1], uy = mom[4 * m + 2], T = mom[4 * m + 3];
  const double A = rho / (2.0 * M_PI * T), inv2T = 0.5 / T, invT = 1.0 / T;
  const double qx = SK ? heat[2 * m] : 0.0, qy = SK ? heat[2 * m + 1] : 0.0;
  const double ska = SK ? P.sk_coef / (rho * T * T) : 0.0;
  const double nv = nu[m], sc = 1.0 / (1.0 + nv);
  Sums2<SK> sm;
  for (int p = threadIdx.x; p < nvel; p += blockDim.x) {
    const double vx = vnode(P.vmin, P.dv, p % N), vy = vnode(P.vmin, P.dv, p / N);
    const double cx = vx - ux, cy = vy - uy;
    double E = A * exp(-(cx * cx + cy * cy) * inv2T), Eg = 0.5 * T * E;
    if (SK) shakhov2(ska, qx, qy, T, invT, cx, cy, E, E, Eg);
    const double2 o = st[(size_t)m * nvel + p];
    const double fn = (o.x + nv * E) * sc;
    const double gn = (o.y + nv * Eg) * sc;
    for (int t = b; t < e; ++t) st[(size_t)G.mem[t] * nvel + p] = make_double2(fn, gn);
    sm.add(vx, vy, fn, gn);
  }
  sm.reduce([&](double v) { return block_sum4(v, lds); });
  if (threadIdx.x == 0) {
    double mo[4], hq[2];
    sm.finish(P.w, mo, hq);
    for (int t = b; t < e; ++t) {
      const int k = G.mem[t];
      for (int i = 0; i < 4; ++i) mom[4 * k + i] = mo[i];
      if (SK) { heat[2 * k] = hq[0]; heat[2 * k + 1] = hq[1]; }
    }
    mpart[q] = G.scv[m] * mo[0];   // mass of the new value (replaces the transported one)
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
  P.shakhov = ctx->cfg.model == CC_MODEL_SHAKHOV;
  P.implicit = 0;
  P.sk_coef = (1.0 - ctx->cfg.prandtl) / 5.0;
  return P;
}

// =====================================================================
// Moving body (seven-step summary of Section 3.3.4).  With G0 the geometry
// at t^n and G1 the geometry at t^{n+1} (built inside a box around the body
// from the pose at t^{n+1}), one step is:
//   merge over the control volumes sigma^n of G0 (eq. FusionDD),
//   k_steplist2d: the control volume of t^n that each cell of t^{n+1}
//     receives from (cells appearing at t^{n+1} hop across their largest
//     new edge into a cell of sigma^n), the control volumes whose update
//     differs from a plain gas cell (cut, merged, receiving an appearing
//     cell, or changing area), and the cells left holding stale values,
//   k_genstep2d: those control volumes, with the area ratio S^n/S^{n+1,*}
//     of eq. (ExSchemeDD) and the wall velocity of eq. (uwDD) at t^n,
//   k_step2d: every other cell (plain gas cell at both times),
//   k_rigid2d: force and torque of t^n, then the body velocity at t^{n+1}
//     (eq. motionDD_vit) and the pose at t^{n+1} (eq. motionDD_posit).
// =====================================================================

struct MoveArgs {
  Geo2D G0, G1;
  int* skind;
  int* target;
  int* rcnt;
  int* age;
  int* gl;
  int* gptr;
  int* gmem;
  int* gcount;
  Box2D bx;
};

// pose at t^{n+1} from the state at t^n (position updated with the old
// velocity, eq. motionDD_posit)
__global__ void k_pose_next2d(const double* __restrict__ body, double* __restrict__ pose,
                              double dt) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    pose[0] = body[0] + dt * body[3];
    pose[1] = body[1] + dt * body[4];
    pose[2] = body[2] + dt * body[5];
  }
}

__global__ void __launch_bounds__(1024) k_steplist2d(MoveArgs M) {
  __shared__ int sh[1024];
  const Geo2D& G0 = M.G0;
  const Geo2D& G1 = M.G1;
  const int nx = G0.nx;
  const int nbox = M.bx.ni * M.bx.nj;
  auto cell = [&](int u) { return (M.bx.j0 + u / M.bx.ni) * nx + M.bx.i0 + u % M.bx.ni; };
  auto in_box = [&](int c) {
    const int i = c % nx - M.bx.i0, j = c / nx - M.bx.j0;
    return i >= 0 && i < M.bx.ni && j >= 0 && j < M.bx.nj;
  };
  const int t = threadIdx.x, nth = blockDim.x;
  int bad = 0;
  // receiving control volume of every cell of t^{n+1} (one cell per thread
  // and round)
  for (int u = t; u < nbox; u += nth) {
    const int c = cell(u);
    int tg = G0.master[c];
    if (tg < 0 && G1.type[c] != TYPE_SOLID) {
      // appearing cell: hop across its largest edge of t^{n+1} into sigma^n
      int i = c % nx, j = c / nx, hops = 0;
      while (G0.master[j * nx + i] < 0) {
        if (hops == kHopCap || !hop2d(G1, i, j)) { bad = 1; break; }
        ++hops;
      }
      tg = G0.master[j * nx + i];
    }
    M.target[c] = tg;
    M.rcnt[c] = 0;
  }
  __syncthreads();
  // receivers other than the master itself, counted per master (integer
  // atomics: the count does not depend on their order)
  for (int u = t; u < nbox; u += nth) {
    const int c = cell(u);
    const int tg = M.target[c];
    if (tg >= 0 && tg != c && in_box(tg)) atomicAdd(&M.rcnt[tg], 1);
  }
  __syncthreads();
  // per-cell kinds and the control volumes that need the general update, in
  // ascending cell order (kScanPer consecutive cells per thread, a block scan
  // per round)
  int carry = 0;
  for (int base = 0; base < nbox; base += nth * kScanPer) {
    int c[kScanPer], general[kScanPer], cnt = 0;
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
      const int u = base + t * kScanPer + e;
      c[e] = 0;
      general[e] = 0;
      if (u < nbox) {
        c[e] = cell(u);
        const int tg = M.target[c[e]];
        int kind = KIND_SOLID;
        if (tg == c[e]) {
          general[e] = G0.kind[tg] != KIND_REGULAR || load_l2(&M.rcnt[tg]) != 0 || G1.type[tg] != TYPE_GAS;
          kind = general[e] ? KIND_IRREGULAR : KIND_REGULAR;
        } else if (tg >= 0) {
          kind = KIND_MEMBER;
        }
        M.skind[c[e]] = kind;
      }
      cnt += general[e];
    }
    int tot;
    int w = carry + block_scan_excl(cnt, sh, &tot);
#pragma unroll
    for (int e = 0; e < kScanPer; ++e)
      if (general[e]) M.gl[w++] = c[e];
    carry += tot;
  }
  const int tot_gen = carry;
  // then the cells to zero: solid at t^n and t^{n+1} but not at t^{n-1}, so
  // their entry in the output buffer (the state of t^{n-1}) is stale; ages
  carry = 0;
  for (int base = 0; base < nbox; base += nth * kScanPer) {
    int c[kScanPer], zero[kScanPer], cnt = 0;
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
      const int u = base + t * kScanPer + e;
      c[e] = 0;
      zero[e] = 0;
      if (u < nbox) {
        c[e] = cell(u);
        const int a = M.age[c[e]];
        const bool solid = G1.type[c[e]] == TYPE_SOLID;
        zero[e] = solid && a == 1;
        M.age[c[e]] = solid ? min(a + 1, 2) : 0;
      }
      cnt += zero[e];
    }
    int tot;
    int w = tot_gen + carry + block_scan_excl(cnt, sh, &tot);
#pragma unroll
    for (int e = 0; e < kScanPer; ++e)
      if (zero[e]) M.gl[w++] = -1 - c[e];
    carry += tot;
  }
  const int tot_zero = carry;
  __syncthreads();
  // receivers of each general control volume: CSR pointers by a chunked
  // scan, then the cells placed through atomic cursors and each list sorted
  // into ascending cell order
  carry = 0;
  for (int base = 0; base < tot_gen; base += nth) {
    const int q = base + t;
    int cnt = 0;
    if (q < tot_gen) {
      cnt = 1 + load_l2(&M.rcnt[M.gl[q]]);
      if (cnt > kMaxMembers) bad |= 2;
    }
    int tot;
    const int ex = block_scan_excl(cnt, sh, &tot);
    if (q < tot_gen) M.gptr[q] = carry + ex;
    carry += tot;
  }
  if (t == 0) M.gptr[tot_gen] = carry;
  __syncthreads();   // every count is read before it becomes a cursor
  for (int q = t; q < tot_gen; q += nth) M.rcnt[M.gl[q]] = M.gptr[q];
  __syncthreads();
  for (int u = t; u < nbox; u += nth) {
    const int c = cell(u), tg = M.target[c];
    if (tg >= 0 && in_box(tg) && M.skind[tg] == KIND_IRREGULAR) M.gmem[atomicAdd(&M.rcnt[tg], 1)] = c;
  }
  __syncthreads();
  for (int q = t; q < tot_gen; q += nth) {
    const int b = M.gptr[q], e = M.gptr[q + 1];
    if (load_l2(&M.rcnt[M.gl[q]]) != e) bad |= 4;
    sort_cells(M.gmem + b, e - b);
  }
  if (t == 0) {
    M.gcount[0] = tot_gen + tot_zero;
    M.gcount[2] = tot_gen;
  }
  if (bad) atomicOr(&M.gcount[1], bad);
}

// One general control volume (or one stale cell to zero) per block.
template <bool SK>
__device__ void general_cv(const MoveArgs& M, const double2* __restrict__ in,
                           double2* __restrict__ out, double* __restrict__ mom, double* __restrict__ heat,
                           double* __restrict__ fslot, double* __restrict__ mpart,
                           const double* __restrict__ body, const StepParams& P, int q,
                           CvStage& cs) {
  const Geo2D& G0 = M.G0;
  const Geo2D& G1 = M.G1;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int nvel = G0.nvel;
  const int e0 = M.gl[q];
  if (e0 < 0) {
    const int c = -1 - e0;
    for (int p = tid; p < nvel; p += nth) out[(size_t)c * nvel + p] = make_double2(0.0, 0.0);
    if (tid == 0) { fslot[3 * q] = 0.0; fslot[3 * q + 1] = 0.0; fslot[3 * q + 2] = 0.0; *mpart = 0.0; }
    return;
  }
  const int m = e0;
  const int b = M.gptr[q];
  // more receivers than supported is reported by k_steplist2d; never index past the arrays
  const int nm = min(M.gptr[q + 1] - b, kMaxMembers);
  const double rho = mom[4 * m + 0], ux = mom[4 * m + 1], uy = mom[4 * m + 2], T = mom[4 * m + 3];
  const double dtau = P.tau_coef > 0.0 ? P.dt * rho / P.tau_coef : 0.0;
  const double qx = SK ? heat[2 * m] : 0.0, qy = SK ? heat[2 * m + 1] : 0.0;
  const double Sn = G0.scv[m];
  double Snew = 0.0;
  for (int t = 0; t < nm; ++t) Snew += G1.sbar[M.gmem[b + t]];
  if (tid < nm) {
    const int k = M.gmem[b + tid];
    cs.dst[tid] = out + (size_t)k * nvel;
    cs.live[tid] = G1.type[k] != TYPE_SOLID && Snew > 0.0;
  }
  const double ratio = Snew > 0.0 ? Sn / Snew : 0.0;
  const double dts = Snew > 0.0 ? P.dt / Snew : 0.0;
  Sums2<SK> sm;
  double Fx, Fy, Tq;
  cv_update<SK>(cs, G0, M.gmem + b, nm, in, in + (size_t)m * nvel, body, P, rho, ux, uy, T, qx, qy,
                dtau, ratio, dts, sm, Fx, Fy, Tq);
  if (tid == 0) {
    double mo[4], hq[2];
    sm.finish(P.w, mo, hq);
    for (int t = 0; t < nm; ++t) {
      const int k = M.gmem[b + t];
      for (int i = 0; i < 4; ++i) mom[4 * k + i] = mo[i];
      if (SK) { heat[2 * k] = hq[0]; heat[2 * k + 1] = hq[1]; }
    }
    fslot[3 * q + 0] = Fx;
    fslot[3 * q + 1] = Fy;
    fslot[3 * q + 2] = Tq;
    *mpart = Snew > 0.0 ? Snew * mo[0] : 0.0;
  }
}

__global__ void __launch_bounds__(256) k_genstep2d(MoveArgs M, const double2* __restrict__ in,
                                                   double2* __restrict__ out,
                                                   double* __restrict__ mom,
                                                   double* __restrict__ heat,
                                                   double* __restrict__ fslot,
                                                   double* __restrict__ mpart, int ntiles,
                                                   const double* __restrict__ body, StepParams P) {
  __shared__ CvStage cs;
  const int cnt = M.gcount[0];
  for (int q = blockIdx.x; q < cnt; q += gridDim.x) {
    if (P.shakhov) general_cv<true>(M, in, out, mom, heat, fslot, mpart + ntiles + q, body, P, q, cs);
    else general_cv<false>(M, in, out, mom, nullptr, fslot, mpart + ntiles + q, body, P, q, cs);
  }
}

// Force and torque of t^n in fixed order (the general control volumes'
// slots), then the rigid body: pose at t^{n+1} and, for free rotation, the
// angular velocity at t^{n+1} from the torque of t^n (eq. motionDD_vit).
// The number of general entries of this step is kept in gcount[4 + par]
// for the mass row, since the step lists of the next step may be built
// before that row is reduced.
__global__ void __launch_bounds__(256) k_rigid2d(int* __restrict__ gcount, int par,
                                                 const double* __restrict__ fslot,
                                                 double* __restrict__ body,
                                                 const double* __restrict__ pose, double dt,
                                                 double inv_inertia, int free_rotation,
                                                 double* force_row) {
  __shared__ double lds[8];
  const int ng = gcount[0];
  double fx = 0.0, fy = 0.0, tq = 0.0;
  for (int q = threadIdx.x; q < ng; q += blockDim.x) {
    fx += fslot[3 * q]; fy += fslot[3 * q + 1]; tq += fslot[3 * q + 2];
  }
  fx = block_sum4(fx, lds);
  fy = block_sum4(fy, lds); tq = block_sum4(tq, lds);
  if (threadIdx.x == 0) {
    if (force_row) { force_row[0] = fx; force_row[1] = fy; force_row[2] = tq; }
    body[0] = pose[0]; body[1] = pose[1]; body[2] = pose[2];
    if (free_rotation) body[5] = body[5] + dt * tq * inv_inertia;
    gcount[4 + par] = ng;
  }
}

// mass of t^{n+1}: the regular tiles' partials, then the general entries'
__global__ void __launch_bounds__(256) k_moving_mass2d(const int* __restrict__ gcount, int par,
                                                       const double* __restrict__ mpart, int ntiles,
                                                       double* mass_row) {
  __shared__ double lds[8];
  const int ng = gcount[4 + par];
  double ms = 0.0;
  for (int t = threadIdx.x; t < ntiles + ng; t += blockDim.x) ms += mpart[t];
  ms = block_sum4(ms, lds);
  if (threadIdx.x == 0) mass_row[0] = ms;
}


// =====================================================================
// Batched step: many independent instances (each its own grid, velocity
// grid, Kn, T_w, Mach) advanced together.  One kernel walks the cut/merged
// control volumes of every instance, and one kernel per velocity-grid size
// walks the regular-cell tiles of every instance of that size, in an
// XCD-aware order; a step is captured once as a hipGraph.
// =====================================================================
struct BatchInst {
  Geo2D G;
  FusedArgs A;
  StepParams P;
  TileArgs T;
};

template <int NCH>
__global__ void __launch_bounds__(256) k_batch_tiles2d(const BatchInst* __restrict__ D,
                                                       const int2* __restrict__ items, int nitems,
                                                       int nitems_pad) {
  __shared__ double lds[8];
  // the lower halves exchanged through LDS as in the single-instance kernel
  constexpr bool kX = NCH <= 16;
  __shared__ d2v xlo[kX ? kTileW * NCH * kWave : 1];
  const int b = blockIdx.x;
  const int per = nitems_pad / 8;
  const int w = (b % 8) * per + b / 8;
  if (w >= nitems) return;
  const int2 it = items[w];
  const int inst = __builtin_amdgcn_readfirstlane(it.x);
  const int tile = __builtin_amdgcn_readfirstlane(it.y);
  regular_tile<NCH, false, false>(D[inst].T, D[inst].P, tile, lds, kX ? xlo : nullptr);
}

__global__ void __launch_bounds__(256) k_batch_cut2d(const BatchInst* __restrict__ D,
                                                     const int2* __restrict__ items, int nitems) {
  __shared__ CvStage cs;
  const int w = blockIdx.x;
  if (w >= nitems) return;
  const int2 it = items[w];
  const int inst = __builtin_amdgcn_readfirstlane(it.x);
  const int q = __builtin_amdgcn_readfirstlane(it.y);
  const Geo2D G = D[inst].G;
  const FusedArgs A = D[inst].A;
  cut_cv<false>(G, A.in, A.out, A.mom, nullptr, A.fslot, A.mpart + A.ntiles + q, A.body, D[inst].P, q, cs);
}

typedef void (*batch_tiles_fn)(hipStream_t, const BatchInst*, const int2*, int);

template <int NCH>
void launch_batch_tiles(hipStream_t st, const BatchInst* D, const int2* items, int n) {
  const int pad = (n + 7) / 8 * 8;
  k_batch_tiles2d<NCH><<<pad, 256, 0, st>>>(D, items, n, pad);
}

batch_tiles_fn pick_batch_tiles(int nch) {
  switch (nch) {
    case 1: return launch_batch_tiles<1>;
    case 2: return launch_batch_tiles<2>;
    case 3: return launch_batch_tiles<3>;
    case 4: return launch_batch_tiles<4>;
    case 5: return launch_batch_tiles<5>;
    case 6: return launch_batch_tiles<6>;
    case 7: return launch_batch_tiles<7>;
    case 8: return launch_batch_tiles<8>;
    case 9: return launch_batch_tiles<9>;
    case 10: return launch_batch_tiles<10>;
    case 11: return launch_batch_tiles<11>;
    case 12: return launch_batch_tiles<12>;
    case 13: return launch_batch_tiles<13>;
    case 14: return launch_batch_tiles<14>;
    case 16: return launch_batch_tiles<16>;
    default: return nullptr;
  }
}

typedef void (*fused_fn)(const cc_ctx*, dim3, const FusedArgs&, const StepParams&);

template <int NCH, bool SK, bool IM>
void launch_fused(const cc_ctx* ctx, dim3 grid, const FusedArgs& A, const StepParams& P) {
  if constexpr (IM) k_step2d_im<NCH, SK><<<grid, 256, 0, ctx->stream>>>(ctx->g2, A, P);
  else k_step2d<NCH, SK><<<grid, 256, 0, ctx->stream>>>(ctx->g2, A, P);
}

// fused semi-implicit variants for the velocity grids of the workloads
// (N <= 32); larger grids take the separate relaxation pass
template <bool SK>
fused_fn pick_fused_im(int nch) {
  switch (nch) {
    case 1: return launch_fused<1, SK, true>;
    case 2: return launch_fused<2, SK, true>;
    case 3: return launch_fused<3, SK, true>;
    case 4: return launch_fused<4, SK, true>;
    case 5: return launch_fused<5, SK, true>;
    case 6: return launch_fused<6, SK, true>;
    case 7: return launch_fused<7, SK, true>;
    case 8: return launch_fused<8, SK, true>;
    default: return nullptr;
  }
}

template <bool SK>
fused_fn pick_fused_sk(int nch) {
  switch (nch) {
    case 1: return launch_fused<1, SK, false>;
    case 2: return launch_fused<2, SK, false>;
    case 3: return launch_fused<3, SK, false>;
    case 4: return launch_fused<4, SK, false>;
    case 5: return launch_fused<5, SK, false>;
    case 6: return launch_fused<6, SK, false>;
    case 7: return launch_fused<7, SK, false>;
    case 8: return launch_fused<8, SK, false>;
    case 9: return launch_fused<9, SK, false>;
    case 10: return launch_fused<10, SK, false>;
    case 11: return launch_fused<11, SK, false>;
    case 12: return launch_fused<12, SK, false>;
    case 13: return launch_fused<13, SK, false>;
    case 14: return launch_fused<14, SK, false>;
    case 16: return launch_fused<16, SK, false>;
    case 18: return launch_fused<18, SK, false>;
    case 20: return launch_fused<20, SK, false>;
    case 24: return launch_fused<24, SK, false>;
    case 28: return launch_fused<28, SK, false>;
    case 32: return launch_fused<32, SK, false>;
    default: return nullptr;
  }
}

fused_fn pick_fused(int nch, bool sk = false, bool im = false) {
  if (im) return sk ? pick_fused_im<true>(nch) : pick_fused_im<false>(nch);
  return sk ? pick_fused_sk<true>(nch) : pick_fused_sk<false>(nch);
}

// rows of the velocity grid with v_y < 0 (the lower half of a cell row)
int split_rows(const cc_ctx* ctx) {
  int s = 0;
  for (int p = 0; p < ctx->N; ++p) s += (ctx->cfg.vmin + (p + 0.5) * ctx->dv) < 0.0;
  return s;
}

int chunks_per_half(const cc_ctx* ctx) {
  int s = split_rows(ctx);
  int rows = s > ctx->N - s ? s : ctx->N - s;
  return (rows * ctx->N + 63) / 64;
}

}  // namespace

bool regular_supported_2d(int nvel) {
  // the half-row window holds at most 32 chunks of 64 velocities per half
  int n = (int)lround(sqrt((double)nvel));
  return pick_fused((((n + 1) / 2) * n + 63) / 64) != nullptr;
}

hipError_t launch_force_only_2d(cc_ctx* ctx, double* out4) {
  StepParams P = params2d(ctx);
  P.write_state = 0;
  const double2* in = (const double2*)ctx->state[ctx->cur];
  k_cut_force2d<<<kListBlocks, 256, 0, ctx->stream>>>(ctx->g2, in, ctx->s.mom, ctx->s.fslot,
                                                      ctx->s.body, P);
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
  StepParams P = params2d(ctx);
  prof_begin(ctx, 3);
  k_merge2d<<<kListBlocks, 256, 0, ctx->stream>>>(ctx->g2, (double2*)ctx->state[ctx->cur],
                                                  ctx->s.mom, ctx->s.heat, P);
  prof_end(ctx, 3);
  return hipGetLastError();
}

hipError_t launch_moments_all_2d(cc_ctx* ctx, bool regular_only) {
  StepParams P = params2d(ctx);
  k_mom2d<<<(ctx->ncell + 3) / 4, 256, 0, ctx->stream>>>(
      ctx->g2, (const double2*)ctx->state[ctx->cur], ctx->s.mom, ctx->s.heat, P, regular_only ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_moments_out_2d(cc_ctx* ctx, double* out) {
  StepParams P = params2d(ctx);
  k_momout2d<<<(ctx->ncell + 3) / 4, 256, 0, ctx->stream>>>(
      ctx->g2, (const double2*)ctx->state[ctx->cur], out, P);
  return hipGetLastError();
}

// One semi-implicit step (ImpSchemeDD, fixed body); row (nullable) = force,
// torque and mass of the state entering the step.
hipError_t launch_imex_step_2d(cc_ctx* ctx, double* row) {
  hipStream_t s = ctx->stream;
  StepParams P = params2d(ctx);
  unsigned int* ticket = reinterpret_cast<unsigned int*>(ctx->s.red + 4 * kRedBlocks);
  if (row)   // mass of the state at t^n from its moments
    k_reduce2d<<<kRedBlocks, 256, 0, s>>>(ctx->g2, ctx->s.mom, ctx->s.fslot, ctx->s.red, ticket,
                                          nullptr, row + 3);
  k_imex_nu2d<<<(ctx->ncell + 255) / 256, 256, 0, s>>>(ctx->g2, ctx->s.mom, ctx->s.nu, P.dt, P.tau_coef);
  const int par = ctx->step_parity;
  // transport: the step kernels without relaxation (the force of t^n is
  // computed by the cut kernel into this parity's slots)
  hipError_t e = launch_step_2d_fused(ctx, false, nullptr, nullptr, false, false);
  if (e != hipSuccess) return e;
  if (row) {
    const double* fs = ctx->s.fslot + (par ? 3 * (size_t)ctx->ncell : 0);
    k_reduce2d<<<kRedBlocks, 256, 0, s>>>(ctx->g2, ctx->s.mom, fs, ctx->s.red, ticket, row, nullptr);
  }
  if (ctx->cfg.maxwellian == CC_MAXW_CONSERVATIVE && P.tau_coef > 0.0) {
    prof_begin(ctx, 4);
    k_newton2d<<<(ctx->ncell + 255) / 256, 256, 0, s>>>(ctx->g2, ctx->s.mom, P.vmin, P.dv);
    prof_end(ctx, 4);
  }
  prof_begin(ctx, 5);
  k_relax2d<<<(ctx->ncell + 3) / 4, 256, 0, s>>>(ctx->g2, (double2*)ctx->state[ctx->cur], ctx->s.mom,
                                                 ctx->s.heat, ctx->s.nu, ctx->s.mom2, ctx->s.heat2, P);
  prof_end(ctx, 5);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (P.shakhov) {
    e = hipMemcpyAsync(ctx->s.heat, ctx->s.heat2, (size_t)ctx->ncell * 2 * sizeof(double),
                       hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipMemcpyAsync(ctx->s.mom, ctx->s.mom2, (size_t)ctx->ncell * 4 * sizeof(double),
                        hipMemcpyDeviceToDevice, s);
}

bool imex_fused_2d(const cc_ctx* ctx) {
  return ctx->cfg.maxwellian != CC_MAXW_CONSERVATIVE &&
         pick_fused(chunks_per_half(ctx), ctx->cfg.model == CC_MODEL_SHAKHOV, true) != nullptr;
}

// One semi-implicit step with the direct equilibrium (ImpSchemeDD): the
// streaming kernel relaxes the regular cells right after their transport;
// the cut kernel only transports, and the cut and merged control volumes
// are relaxed afterwards (their mass partials replaced by those of the new
// value).  The force and mass rows are reduced as in the explicit step:
// by block 0 of the next step's streaming kernel, and by
// launch_step_2d_flush after the last one.
hipError_t launch_imex_fused_2d(cc_ctx* ctx, bool reduce_prev, double* prev_force_row, double* cur_mass_row) {
  hipStream_t s = ctx->stream;
  StepParams P = params2d(ctx);
  k_imex_nu2d<<<(ctx->ncell + 255) / 256, 256, 0, s>>>(ctx->g2, ctx->s.mom, ctx->s.nu, P.dt, P.tau_coef);
  hipError_t e = launch_step_2d_fused(ctx, reduce_prev, prev_force_row, cur_mass_row, true, true, true);
  if (e != hipSuccess) return e;
  if (ctx->n_irr > 0) {
    const int par = 1 - ctx->step_parity;   // parity of the step just launched
    double* mp = ctx->s.mpart + (par ? (size_t)ctx->s.mpart_cap : 0) + ctx->last_args_ntiles;
    prof_begin(ctx, 5);
    if (P.shakhov)
      k_relax_cut2d<true><<<ctx->n_irr, 256, 0, s>>>(ctx->g2, (double2*)ctx->state[ctx->cur], ctx->s.mom,
                                                      ctx->s.heat, ctx->s.nu, mp, P);
    else
      k_relax_cut2d<false><<<ctx->n_irr, 256, 0, s>>>(ctx->g2, (double2*)ctx->state[ctx->cur], ctx->s.mom,
                                                       nullptr, ctx->s.nu, mp, P);
    prof_end(ctx, 5);
  }
  return hipGetLastError();
}

// mass of the current state into mass_row (no force)
hipError_t launch_mass_2d(cc_ctx* ctx, double* mass_row) {
  k_reduce2d<<<kRedBlocks, 256, 0, ctx->stream>>>(
      ctx->g2, ctx->s.mom, ctx->s.fslot, ctx->s.red,
      reinterpret_cast<unsigned int*>(ctx->s.red + 4 * kRedBlocks), nullptr, mass_row);
  return hipGetLastError();
}

// Tile shape of the regular-cell pass: kTileW columns x seglen rows.
int tile_rows(const cc_ctx* ctx) {
  if (ctx->seglen > 0) return ctx->seglen;
  // Fixed body: ~2 tiles per CU on 256 CUs (as many as are resident at
  // once).  Moving body: ~16 per CU, so that blocks retire all through the
  // streaming kernel and the next step's geometry kernels, queued beside it
  // on the side stream, find free slots early instead of in its tail
  // (ellipse256: 0.79 against 0.92 ms per step).
  const bool moving = ctx->body.motion != CC_MOTION_FIXED && ctx->body.kind != CC_BODY_NONE;
  const int groups = (ctx->nx + kTileW - 1) / kTileW;
  const int target = moving ? 4096 : 512;
  int segs = (target + groups - 1) / groups;
  if (segs < 1) segs = 1;
  int rows = (ctx->ny + segs - 1) / segs;
  return rows < 1 ? 1 : rows;
}

// One step: state[cur] -> state[1-cur].  When diag is requested, this
// launch also reduces the previous step's partials (deferred) into
// diag rows; the last step's are reduced by cc_step through
// launch_step_2d_flush.
hipError_t launch_step_2d_fused(cc_ctx* ctx, bool reduce_prev, double* prev_force_row,
                                double* cur_mass_row, bool record, bool relax, bool implicit) {
  StepParams P = params2d(ctx);
  if (!relax) P.tau_coef = 0.0;   // transport only (first half of the semi-implicit step)
  P.implicit = implicit;          // transport, then the implicit relaxation of the regular cells
  fused_fn fn = pick_fused(chunks_per_half(ctx), P.shakhov, implicit);
  if (!fn) return hipErrorInvalidValue;
  const int par = ctx->step_parity;
  FusedArgs A;
  A.kind = ctx->g2.kind;
  A.in = (const double2*)ctx->state[ctx->cur];
  A.out = (double2*)ctx->state[1 - ctx->cur];
  A.mom = ctx->s.mom;
  A.heat = ctx->s.heat;
  A.body = ctx->s.body;
  A.ngroups = (ctx->nx + kTileW - 1) / kTileW;
  A.seglen = tile_rows(ctx);
  const int nseg = (ctx->ny + A.seglen - 1) / A.seglen;
  A.ntiles = A.ngroups * nseg;
  A.ntiles_pad = (A.ntiles + 7) / 8 * 8;
  A.n_cut = ctx->n_irr;
  A.cut_base = 0;
  A.tile_base = 8;
  A.split = split_rows(ctx);
  const int nparts = A.ntiles + A.n_cut;
  double* fs[2] = {ctx->s.fslot, ctx->s.fslot + 3 * (size_t)ctx->ncell};
  double* mp[2] = {ctx->s.mpart, ctx->s.mpart + (size_t)ctx->s.mpart_cap};
  if (nparts > ctx->s.mpart_cap) return hipErrorInvalidValue;
  A.fslot = fs[par];
  A.mpart = mp[par];
  A.prev_fslot = reduce_prev ? fs[1 - par] : nullptr;
  A.prev_mpart = reduce_prev ? mp[1 - par] : nullptr;
  A.red_force = prev_force_row;
  A.red_mass = cur_mass_row;
  dim3 grid(A.tile_base + A.ntiles_pad);
  if (relax && !implicit && ctx->cfg.maxwellian == CC_MAXW_CONSERVATIVE) {
    prof_begin(ctx, 4);
    k_newton2d<<<(ctx->ncell + 255) / 256, 256, 0, ctx->stream>>>(ctx->g2, ctx->s.mom, P.vmin, P.dv);
    prof_end(ctx, 4);
  }
  // the cut control volumes (disjoint cells, their own partial slots) run on
  // a side stream beside the streaming kernel; serial while profiling
  const bool overlap = A.n_cut > 0 && ctx->side && !ctx->prof.on;
  if (overlap) {
    hipError_t e = hipEventRecord(ctx->fork, ctx->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(ctx->side, ctx->fork, 0);
    if (e != hipSuccess) return e;
    k_cutstep2d<<<A.n_cut, 256, 0, ctx->side>>>(ctx->g2, A, P);
    e = hipEventRecord(ctx->join, ctx->side);
    if (e != hipSuccess) return e;
  } else if (A.n_cut > 0) {
    prof_begin(ctx, 1);
    k_cutstep2d<<<A.n_cut, 256, 0, ctx->stream>>>(ctx->g2, A, P);
    prof_end(ctx, 1);
  }
  prof_begin(ctx, 0);
  fn(ctx, grid, A, P);
  prof_end(ctx, 0);
  if (overlap) {
    hipError_t e = hipStreamWaitEvent(ctx->stream, ctx->join, 0);
    if (e != hipSuccess) return e;
  }
  ctx->last_args_ntiles = A.ntiles;
  ctx->cur = 1 - ctx->cur;
  ctx->step_parity = 1 - par;
  (void)record;
  return hipGetLastError();
}

__global__ void k_moving_init2d(Geo2D G, int* __restrict__ skind0, int* __restrict__ skind1,
                                int* __restrict__ target, int* __restrict__ age) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.ncell) return;
  skind0[c] = G.kind[c];
  skind1[c] = G.kind[c];
  target[c] = G.master[c];
  age[c] = G.type[c] == TYPE_SOLID ? 2 : 0;
}

hipError_t launch_moving_init_2d(cc_ctx* ctx) {
  k_moving_init2d<<<(ctx->ncell + 255) / 256, 256, 0, ctx->stream>>>(ctx->g2, ctx->s.skind, ctx->s.skind2,
                                                                      ctx->s.target, ctx->s.age);
  return hipGetLastError();
}

// Box of cells that can change between t^n and t^{n+1}: the body's extent
// at both times plus a margin covering master searches and receivers.
Box2D moving_box(const cc_ctx* ctx, long long n) {
  const cc_body& b = ctx->body;
  double R = b.axes[0] > b.axes[1] ? b.axes[0] : b.axes[1];
  if (b.kind == CC_BODY_CIRCLE) R = b.axes[0];
  double t0 = n * ctx->dt, t1 = t0 + ctx->dt;
  double vx = b.motion == CC_MOTION_IMPOSED ? b.vel[0] : 0.0;
  double vy = b.motion == CC_MOTION_IMPOSED ? b.vel[1] : 0.0;
  double xa = b.center[0] + vx * t0, xb = b.center[0] + vx * t1;
  double ya = b.center[1] + vy * t0, yb = b.center[1] + vy * t1;
  double xmin = fmin(xa, xb) - R, xmax = fmax(xa, xb) + R;
  double ymin = fmin(ya, yb) - R, ymax = fmax(ya, yb) + R;
  const int margin = 2 * kHopCap + 3;
  int i0 = (int)floor((xmin - ctx->cfg.lo[0]) / ctx->dx) - margin;
  int i1 = (int)ceil((xmax - ctx->cfg.lo[0]) / ctx->dx) + margin;
  int j0 = (int)floor((ymin - ctx->cfg.lo[1]) / ctx->dy) - margin;
  int j1 = (int)ceil((ymax - ctx->cfg.lo[1]) / ctx->dy) + margin;
  i0 = i0 < 0 ? 0 : i0; j0 = j0 < 0 ? 0 : j0;
  i1 = i1 > ctx->nx ? ctx->nx : i1; j1 = j1 > ctx->ny ? ctx->ny : j1;
  return Box2D{i0, j0, i1 - i0, j1 - j0};
}

// Geometry of the time level after step n (body pose from the body state
// of t^n), built into G1 inside the box of step n, and the step lists of
// step n against G0 (the geometry of t^n), written with parity par: the
// per-cell kinds of that parity, the receivers, the general list.
static hipError_t moving_lists_2d(cc_ctx* ctx, hipStream_t st, const Geo2D& G0, Geo2D& G1, long long n,
                                  int par) {
  k_pose_next2d<<<1, 64, 0, st>>>(ctx->s.body, ctx->s.pose, ctx->dt);
  const Box2D bx = moving_box(ctx, n);
  hipStream_t keep = ctx->stream;
  ctx->stream = st;
  hipError_t e = build_geometry_box_2d(ctx, G1, ctx->s.pose, bx);
  ctx->stream = keep;
  if (e != hipSuccess) return e;
  MoveArgs M;
  M.G0 = G0; M.G1 = G1;
  M.skind = par ? ctx->s.skind2 : ctx->s.skind;
  M.target = ctx->s.target; M.rcnt = ctx->s.rcnt; M.age = ctx->s.age;
  M.gl = ctx->s.gl; M.gptr = ctx->s.gptr; M.gmem = ctx->s.gmem; M.gcount = ctx->s.gcount;
  M.bx = bx;
  k_steplist2d<<<1, 1024, 0, st>>>(M);
  return hipGetLastError();
}

// Before the first step of a call: the geometry of t^{n+1} and the step
// lists of step n (profiling slot 4: the geometry rebuild).
hipError_t launch_moving_prologue_2d(cc_ctx* ctx) {
  prof_begin(ctx, 4);
  hipError_t e = moving_lists_2d(ctx, ctx->stream, ctx->g2, ctx->g2n, ctx->nstep, ctx->step_parity);
  prof_end(ctx, 4);
  return e;
}

// One step of a moving body (Section 3.3.4) whose geometry of t^{n+1} and
// step lists were built before.  Main stream: merge over the control volumes
// of t^n, the streaming kernel over the regular cells, the mass of t^{n+1}.
// Beside it (side stream, after the merge): the general control volumes
// (wall condition, area ratio, receivers), the force and torque of t^n and
// the rigid body, then, when another step follows, the geometry of t^{n+2}
// (into the buffer of t^n, which only the general control volumes read) and
// the step lists of step n+1 (the other parity of the kind array).  While
// profiling everything runs on the main stream in the same order.
hipError_t launch_moving_step_2d(cc_ctx* ctx, double* force_row, double* mass_row, bool next) {
  StepParams P = params2d(ctx);
  fused_fn fn = pick_fused(chunks_per_half(ctx), P.shakhov);
  if (!fn) return hipErrorInvalidValue;
  hipStream_t st = ctx->stream;
  const bool overlap = ctx->side && !ctx->prof.on;
  hipStream_t sd = overlap ? ctx->side : st;
  const int par = ctx->step_parity;
  MoveArgs M;
  M.G0 = ctx->g2; M.G1 = ctx->g2n;
  M.skind = par ? ctx->s.skind2 : ctx->s.skind;
  M.target = ctx->s.target; M.rcnt = ctx->s.rcnt; M.age = ctx->s.age;
  M.gl = ctx->s.gl; M.gptr = ctx->s.gptr; M.gmem = ctx->s.gmem; M.gcount = ctx->s.gcount;
  M.bx = moving_box(ctx, ctx->nstep);
  // 2. merge over the control volumes of t^n
  prof_begin(ctx, 3);
  k_merge2d<<<kListBlocks, 256, 0, st>>>(ctx->g2, (double2*)ctx->state[ctx->cur], ctx->s.mom,
                                        ctx->s.heat, P);
  prof_end(ctx, 3);
  FusedArgs A;
  A.kind = M.skind;
  A.in = (const double2*)ctx->state[ctx->cur];
  A.out = (double2*)ctx->state[1 - ctx->cur];
  A.mom = ctx->s.mom;
  A.heat = ctx->s.heat;
  A.body = ctx->s.body;
  A.ngroups = (ctx->nx + kTileW - 1) / kTileW;
  A.seglen = tile_rows(ctx);
  const int nseg = (ctx->ny + A.seglen - 1) / A.seglen;
  A.ntiles = A.ngroups * nseg;
  A.ntiles_pad = (A.ntiles + 7) / 8 * 8;
  A.n_cut = 0;
  A.cut_base = 0;
  A.tile_base = 8;
  A.split = split_rows(ctx);
  double* fs = ctx->s.fslot + (size_t)par * 3 * ctx->ncell;
  double* mp = ctx->s.mpart + (size_t)par * ctx->s.mpart_cap;
  A.fslot = fs;
  A.mpart = mp;
  A.prev_fslot = nullptr;
  A.prev_mpart = nullptr;
  A.red_force = nullptr;
  A.red_mass = nullptr;
  hipError_t e;
  if (overlap) {
    if ((e = hipEventRecord(ctx->fork, st)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(sd, ctx->fork, 0)) != hipSuccess) return e;
  }
  // 4-6. wall condition, scheme and redistribution of the general control
  // volumes; 5/1. force and torque of t^n, body velocity and pose at t^{n+1}
  prof_begin(ctx, 1);
  k_genstep2d<<<kListBlocks, 256, 0, sd>>>(M, A.in, A.out, A.mom, A.heat, fs, mp, A.ntiles, ctx->s.body, P);
  prof_end(ctx, 1);
  const bool free_rot = ctx->body.motion == CC_MOTION_FREE_ROTATION;
  prof_begin(ctx, 2);
  k_rigid2d<<<1, 256, 0, sd>>>(ctx->s.gcount, par, fs, ctx->s.body, ctx->s.pose, ctx->dt,
                               free_rot ? 1.0 / ctx->body.inertia : 0.0, free_rot ? 1 : 0, force_row);
  prof_end(ctx, 2);
  if (overlap && next) {
    // the next step's geometry and lists beside the streaming kernel
    if ((e = moving_lists_2d(ctx, sd, ctx->g2n, ctx->g2, ctx->nstep + 1, 1 - par)) != hipSuccess) return e;
  }
  if (overlap && (e = hipEventRecord(ctx->join, sd)) != hipSuccess) return e;
  // 6. scheme and redistribution of every other (regular) cell
  prof_begin(ctx, 0);
  fn(ctx, dim3(A.tile_base + A.ntiles_pad), A, P);
  prof_end(ctx, 0);
  if (overlap && (e = hipStreamWaitEvent(st, ctx->join, 0)) != hipSuccess) return e;
  if (mass_row) {
    // the mass row off the solver stream: on the side stream once this
    // step's streaming kernel is done (the next step's side work queues
    // behind it; a call's last step, which has no mass row, joins the side
    // stream back before the call returns)
    hipStream_t sm = st;
    if (overlap && next) {
      if ((e = hipEventRecord(ctx->fork, st)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(sd, ctx->fork, 0)) != hipSuccess) return e;
      sm = sd;
    }
    k_moving_mass2d<<<1, 256, 0, sm>>>(ctx->s.gcount, par, mp, A.ntiles, mass_row);
  }
  if (!overlap && next) {
    prof_begin(ctx, 4);
    e = moving_lists_2d(ctx, st, ctx->g2n, ctx->g2, ctx->nstep + 1, 1 - par);
    prof_end(ctx, 4);
    if (e != hipSuccess) return e;
  }
  e = hipGetLastError();
  Geo2D tmp = ctx->g2; ctx->g2 = ctx->g2n; ctx->g2n = tmp;
  ctx->cur = 1 - ctx->cur;
  ctx->step_parity = 1 - par;
  ctx->nstep += 1;
  return e;
}


// ---------------------------------------------------------------------
// batch host side
// ---------------------------------------------------------------------
static FusedArgs fused_args_for(const cc_ctx* ctx, int in_buf, int rows) {
  FusedArgs A;
  A.kind = ctx->g2.kind;
  A.in = (const double2*)ctx->state[in_buf];
  A.out = (double2*)ctx->state[1 - in_buf];
  A.mom = ctx->s.mom;
  A.heat = nullptr;   // batched instances relax with BGK only
  A.body = ctx->s.body;
  A.ngroups = (ctx->nx + kTileW - 1) / kTileW;
  A.seglen = rows;
  const int nseg = (ctx->ny + rows - 1) / rows;
  A.ntiles = A.ngroups * nseg;
  A.ntiles_pad = (A.ntiles + 7) / 8 * 8;
  A.n_cut = ctx->n_irr;
  A.cut_base = 0;
  A.tile_base = 0;
  A.split = split_rows(ctx);
  A.fslot = ctx->s.fslot;
  A.mpart = ctx->s.mpart;
  A.prev_fslot = nullptr;
  A.prev_mpart = nullptr;
  A.red_force = nullptr;
  A.red_mass = nullptr;
  return A;
}

int batch_group_nch(const cc_ctx* ctx) { return chunks_per_half(ctx); }
bool batch_supported_nch(int nch) { return pick_batch_tiles(nch) != nullptr; }

size_t batch_desc_bytes() { return sizeof(BatchInst); }

// Host images of the descriptors (parity 0: each instance reads its current
// buffer; parity 1: the other one) and of the work lists.
void batch_fill(cc_batch* B, std::vector<char>& desc0, std::vector<char>& desc1,
                std::vector<int2>& tiles, std::vector<int2>& cuts) {
  const int n = (int)B->ctx.size();
  desc0.assign(n * sizeof(BatchInst), 0);
  desc1.assign(n * sizeof(BatchInst), 0);
  tiles.clear();
  cuts.clear();
  B->group_off.assign(B->group_nch.size(), 0);
  B->group_cnt.assign(B->group_nch.size(), 0);
  for (size_t g = 0; g < B->group_nch.size(); ++g) {
    B->group_off[g] = (int)tiles.size();
    for (int i = 0; i < n; ++i) {
      cc_ctx* c = B->ctx[i];
      if (batch_group_nch(c) != B->group_nch[g]) continue;
      const int rows = B->group_rows[g] > 0 ? B->group_rows[g] : tile_rows(c);
      for (int par = 0; par < 2; ++par) {
        BatchInst d;
        d.G = c->g2;
        d.A = fused_args_for(c, c->cur ^ par, rows);
        d.P = params2d(c);
        d.T = tile_args(d.G, d.A);
        memcpy((par ? desc1 : desc0).data() + i * sizeof(BatchInst), &d, sizeof(d));
      }
      BatchInst d0;
      memcpy(&d0, desc0.data() + i * sizeof(BatchInst), sizeof(d0));
      for (int t = 0; t < d0.A.ntiles; ++t) tiles.push_back(make_int2(i, t));
    }
    B->group_cnt[g] = (int)tiles.size() - B->group_off[g];
  }
  for (int i = 0; i < n; ++i)
    for (int q = 0; q < B->ctx[i]->n_irr; ++q) cuts.push_back(make_int2(i, q));
}

// launch one batched step (parity 0 or 1) on the batch stream; with side
// streams (graph capture), the cut-cell kernel and each group's tile kernel
// are recorded on their own branch so the graph may run them concurrently
hipError_t batch_launch_step(cc_batch* B, int par, hipStream_t* side, int nside) {
  return batch_launch_desc(B, par ? B->d_desc1 : B->d_desc0, side, nside);
}

// one batched step with the descriptor table D (device)
hipError_t batch_launch_desc(cc_batch* B, const void* Dv, hipStream_t* side, int nside) {
  const BatchInst* D = (const BatchInst*)Dv;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;
  if (nside > 0) {
    hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    hipEventRecord(fork, B->stream);
  }
  int branch = 0;
  auto on_branch = [&]() -> hipStream_t {
    if (nside == 0) return B->stream;
    hipStream_t s = side[branch % nside];
    ++branch;
    hipStreamWaitEvent(s, fork, 0);
    return s;
  };
  auto close_branch = [&](hipStream_t s) {
    if (nside == 0) return;
    hipEvent_t j;
    hipEventCreateWithFlags(&j, hipEventDisableTiming);
    hipEventRecord(j, s);
    joins.push_back(j);
  };
  if (B->ncut > 0) {
    hipStream_t s = on_branch();
    k_batch_cut2d<<<B->ncut, 256, 0, s>>>(D, B->d_cuts, B->ncut);
    close_branch(s);
  }
  for (size_t g = 0; g < B->group_nch.size(); ++g) {
    if (B->group_cnt[g] == 0) continue;
    hipStream_t s = on_branch();
    pick_batch_tiles(B->group_nch[g])(s, D, B->d_tiles + B->group_off[g], B->group_cnt[g]);
    close_branch(s);
  }
  for (hipEvent_t j : joins) hipStreamWaitEvent(B->stream, j, 0);
  hipError_t e = hipGetLastError();
  for (hipEvent_t j : joins) hipEventDestroy(j);
  if (fork) hipEventDestroy(fork);
  return e;
}

// Redirects a host image of an instance's descriptor to other state and
// moment buffers (the steps of the batched adjoint).
void batch_desc_patch(void* desc, const double2* in, double2* out, double* mom) {
  BatchInst& d = *(BatchInst*)desc;
  d.A.in = in;
  d.A.out = out;
  d.A.mom = mom;
  d.T = tile_args(d.G, d.A);
}

// tile kernel of one group only (autotuning)
hipError_t batch_launch_group(cc_batch* B, int g) {
  const BatchInst* D = (const BatchInst*)B->d_desc0;
  pick_batch_tiles(B->group_nch[g])(B->stream, D, B->d_tiles + B->group_off[g], B->group_cnt[g]);
  return hipGetLastError();
}

// one fixed-geometry step with explicit state and moment buffers (no
// reductions): recomputation inside the adjoint
hipError_t launch_step_2d_ptrs(cc_ctx* ctx, const double2* in, double2* out, double* mom) {
  StepParams P = params2d(ctx);
  P.shakhov = 0;   // the adjoint is built for the BGK model only
  fused_fn fn = pick_fused(chunks_per_half(ctx));
  if (!fn) return hipErrorInvalidValue;
  FusedArgs A;
  A.kind = ctx->g2.kind;
  A.in = in;
  A.out = out;
  A.mom = mom;
  A.heat = nullptr;
  A.body = ctx->s.body;
  A.ngroups = (ctx->nx + kTileW - 1) / kTileW;
  A.seglen = tile_rows(ctx);
  const int nseg = (ctx->ny + A.seglen - 1) / A.seglen;
  A.ntiles = A.ngroups * nseg;
  A.ntiles_pad = (A.ntiles + 7) / 8 * 8;
  A.n_cut = ctx->n_irr;
  A.cut_base = 0;
  A.tile_base = 8;
  A.split = split_rows(ctx);
  A.fslot = ctx->s.fslot;
  A.mpart = ctx->s.mpart;
  A.prev_fslot = nullptr;
  A.prev_mpart = nullptr;
  A.red_force = nullptr;
  A.red_mass = nullptr;
  // the cut control volumes beside the streaming kernel, as in the forward step
  const bool overlap = A.n_cut > 0 && ctx->side && !ctx->prof.on;
  if (overlap) {
    hipError_t e = hipEventRecord(ctx->fork, ctx->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(ctx->side, ctx->fork, 0);
    if (e != hipSuccess) return e;
    k_cutstep2d<<<A.n_cut, 256, 0, ctx->side>>>(ctx->g2, A, P);
    e = hipEventRecord(ctx->join, ctx->side);
    if (e != hipSuccess) return e;
  } else if (A.n_cut > 0) {
    k_cutstep2d<<<A.n_cut, 256, 0, ctx->stream>>>(ctx->g2, A, P);
  }
  fn(ctx, dim3(A.tile_base + A.ntiles_pad), A, P);
  if (overlap) {
    hipError_t e = hipStreamWaitEvent(ctx->stream, ctx->join, 0);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// reduce the partials of the step that just ran into its force row and the
// mass row of the state it produced
hipError_t launch_step_2d_flush(cc_ctx* ctx, double* force_row, double* mass_row) {
  const int par = 1 - ctx->step_parity;   // parity of the last launched step
  FusedArgs A{};
  A.ntiles = ctx->last_args_ntiles;
  A.n_cut = ctx->n_irr;
  double* fs[2] = {ctx->s.fslot, ctx->s.fslot + 3 * (size_t)ctx->ncell};
  double* mp[2] = {ctx->s.mpart, ctx->s.mpart + (size_t)ctx->s.mpart_cap};
  A.prev_fslot = fs[par];
  A.prev_mpart = mp[par];
  A.red_force = force_row;
  A.red_mass = mass_row;
  prof_begin(ctx, 2);
  k_final_reduce2d<<<1, 256, 0, ctx->stream>>>(ctx->g2, A);
  prof_end(ctx, 2);
  return hipGetLastError();
}


}  // namespace ccdvm
