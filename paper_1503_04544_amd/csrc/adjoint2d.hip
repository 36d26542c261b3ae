// Hand-written adjoint of the fixed-geometry 2D step (not in the paper: the
// transpose of the scheme of Section 3.3 written out term by term), and the
// checkpointed driver that returns the gradient of the drag or the torque of
// the final state with respect to the wall temperature, the Knudsen number
// and the inflow Mach number.
//
// Notation.  x^n is the merged state entering step n; Lambda^{n+1}_m is the
// sensitivity of the objective to the value that control volume m writes to
// its members at step n.  The kernels store mu_k = Lambda_{master(k)} / S_m
// at every member cell k (zero in solid cells), so that an upwind cell
// gathers its downwind neighbours' sensitivities as a plain stencil:
//   Lambda^n_m = (1 - beta) Lambda + (BGK Jacobian)^T Lambda
//              - dt/S_m sum_edges L c+ Lambda          (own outflow)
//              + dt sum_edges L c+ mu_downwind          (inflow into the neighbour)
//              + wall terms (own outflow, rank one through phi_w).
// beta = dt rho / kappa; the Maxwellian's Jacobian goes through (rho, rho u,
// E) with four reductions per cell of Lambda against dE/d(rho, u, T).
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <vector>

#include "ccdvm_impl.h"

// Contraction off: the adjoint kernel bodies are inlined into the
// single-instance and the batched kernels, and each expression must round
// the same way in both, so that a batched gradient equals the
// single-instance one bit for bit.
#pragma clang fp contract(off)

namespace ccdvm {
namespace {

constexpr int kWave = 64;

__device__ inline double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// sum over the 4 waves of a 256-thread block, in wave order
__device__ inline double bsum(double v, double* lds) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

__device__ inline double vnd(double vmin, double dv, int idx) { return vmin + (idx + 0.5) * dv; }

struct AdjParams {
  double vmin, dv, w, dt;
  double kappa;      // tau = kappa / rho; 0: no collisions
  double kn;
  double t_wall;
  double rho_in, ux_in, uy_in, t_in;   // farfield Maxwellian
  int objective;     // 0 drag, 1 torque
};

struct AdjBufs {
  const double2* x;      // x^n (merged state entering the step)
  const double* mom;     // rho, ux, uy, T of x^n per cell
  const double2* mu_in;  // mu^{n+1}
  double2* mu_out;       // mu^n
  double* part;          // per-block partials (accumulated across steps): T_w, Kn, ux, uy
  const double* body;    // body state (centre for the torque arm)
};

__device__ inline double maxw(double rho, double ux, double uy, double T, double vx, double vy) {
  const double cx = vx - ux, cy = vy - uy;
  return rho / (2.0 * M_PI * T) * exp(-(cx * cx + cy * cy) / (2.0 * T));
}

// reductions of Lambda against the derivatives of the relaxation term:
// A = (A_rho, A_px, A_py, A_E) in (rho, rho u, E) and C = sum Lambda.(Q - x)
struct BgkSums { double Ar, Apx, Apy, Ae, C; };

__device__ inline void bgk_terms(double rho, double ux, double uy, double T, double vx, double vy,
                                 double lf, double lg, double f, double g, double* s) {
  const double cx = vx - ux, cy = vy - uy, c2 = cx * cx + cy * cy;
  const double E = maxw(rho, ux, uy, T, vx, vy);
  const double dEr = E / rho, dEux = E * cx / T, dEuy = E * cy / T;
  const double dET = E * (c2 / (2.0 * T * T) - 1.0 / T);
  s[0] += lf * dEr + lg * 0.5 * T * dEr;
  s[1] += lf * dEux + lg * 0.5 * T * dEux;
  s[2] += lf * dEuy + lg * 0.5 * T * dEuy;
  s[3] += lf * dET + lg * (0.5 * E + 0.5 * T * dET);
  s[4] += lf * (E - f) + lg * (0.5 * T * E - g);
}

__device__ inline BgkSums chain(double rho, double ux, double uy, double T, const double* s) {
  const double u2 = ux * ux + uy * uy;
  BgkSums b;
  b.Ar = s[0] + s[1] * (-ux / rho) + s[2] * (-uy / rho) + s[3] * (u2 - 3.0 * T) / (3.0 * rho);
  b.Apx = s[1] / rho + s[3] * (-2.0 * ux / (3.0 * rho));
  b.Apy = s[2] / rho + s[3] * (-2.0 * uy / (3.0 * rho));
  b.Ae = s[3] * 2.0 / (3.0 * rho);
  b.C = s[4];
  return b;
}

// ---------------------------------------------------------------------
// regular gas cells: one wave per cell
// ---------------------------------------------------------------------
// blk: the block's index among the instance's regular blocks (4 cells each)
__device__ inline void adj_regular_body(const Geo2D& G, const AdjBufs& B, const AdjParams& P, int blk,
                                        double (*lds)[4]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blk * 4 + wave;
  double pk = 0.0, pux = 0.0, puy = 0.0;
  if (c < G.ncell && G.kind[c] == KIND_REGULAR) {
    const int nx = G.nx, ny = G.ny, N = G.N, nvel = G.nvel;
    const int i = c % nx, j = c / nx;
    const double S = G.dx * G.dy;
    const double rho = B.mom[4 * c], ux = B.mom[4 * c + 1], uy = B.mom[4 * c + 2], T = B.mom[4 * c + 3];
    const bool collide = P.kappa > 0.0;
    const double beta = collide ? P.dt * rho / P.kappa : 0.0;
    const double2* mu = B.mu_in + (size_t)c * nvel;
    const double2* xc = B.x + (size_t)c * nvel;
    BgkSums A{0, 0, 0, 0, 0};
    if (collide) {
      double s[5] = {0, 0, 0, 0, 0};
      for (int p = lane; p < nvel; p += kWave) {
        const double2 m = mu[p], x = xc[p];
        bgk_terms(rho, ux, uy, T, vnd(P.vmin, P.dv, p % N), vnd(P.vmin, P.dv, p / N), S * m.x, S * m.y,
                  x.x, x.y, s);
      }
      for (int k = 0; k < 5; ++k) s[k] = wsum(s[k]);
      A = chain(rho, ux, uy, T, s);
      pk = A.C * (-beta / P.kn);
    }
    const double ca = P.dt / G.dx, cb = P.dt / G.dy;
    const double2* xr = i + 1 < nx ? mu + nvel : nullptr;
    const double2* xl = i > 0 ? mu - nvel : nullptr;
    const double2* yu = j + 1 < ny ? mu + (size_t)nx * nvel : nullptr;
    const double2* yd = j > 0 ? mu - (size_t)nx * nvel : nullptr;
    double2* out = B.mu_out + (size_t)c * nvel;
    for (int p = lane; p < nvel; p += kWave) {
      const double vx = vnd(P.vmin, P.dv, p % N), vy = vnd(P.vmin, P.dv, p / N);
      const double a = ca * fabs(vx), b = cb * fabs(vy);
      const double2 m = mu[p];
      // downwind neighbours (none past an outer face: the farfield is fixed)
      const double2* dx_ = vx > 0.0 ? xr : xl;
      const double2* dy_ = vy > 0.0 ? yu : yd;
      const double2 mdx = dx_ ? dx_[p] : make_double2(0.0, 0.0);
      const double2 mdy = dy_ ? dy_[p] : make_double2(0.0, 0.0);
      double of = (1.0 - beta - a - b) * m.x + a * mdx.x + b * mdy.x;
      double og = (1.0 - beta - a - b) * m.y + a * mdx.y + b * mdy.y;
      if (collide) {
        of += (beta * P.w * (A.Ar + A.Apx * vx + A.Apy * vy + A.Ae * 0.5 * (vx * vx + vy * vy)) +
               P.dt * P.w / P.kappa * A.C) / S;
        og += beta * P.w * A.Ae / S;
      }
      out[p] = make_double2(of, og);
      // farfield faces upwind of the cell: d ghost / d u
      const bool ghost_x = (vx > 0.0 && i == 0) || (vx < 0.0 && i == nx - 1);
      const bool ghost_y = (vy > 0.0 && j == 0) || (vy < 0.0 && j == ny - 1);
      if (ghost_x || ghost_y) {
        const double M = maxw(P.rho_in, P.ux_in, P.uy_in, P.t_in, vx, vy);
        const double coef = (ghost_x ? P.dt * G.dy * fabs(vx) : 0.0) + (ghost_y ? P.dt * G.dx * fabs(vy) : 0.0);
        const double t = coef * (m.x + 0.5 * P.t_in * m.y) * M / P.t_in;
        pux += t * (vx - P.ux_in);
        puy += t * (vy - P.uy_in);
      }
    }
  }
  // pk is one value per cell, identical on every lane; the farfield terms are per lane
  pux = wsum(pux);
  puy = wsum(puy);
  if (lane == 0) { lds[wave][0] = pk; lds[wave][1] = pux; lds[wave][2] = puy; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* pt = B.part + 4 * (size_t)blk;
    pt[1] += ((lds[0][0] + lds[1][0]) + lds[2][0]) + lds[3][0];
    pt[2] += ((lds[0][1] + lds[1][1]) + lds[2][1]) + lds[3][1];
    pt[3] += ((lds[0][2] + lds[1][2]) + lds[2][2]) + lds[3][2];
  }
}

__global__ void __launch_bounds__(256) k_adj_regular2d(Geo2D G, AdjBufs B, AdjParams P) {
  __shared__ double lds[4][4];
  adj_regular_body(G, B, P, blockIdx.x, lds);
}

// ---------------------------------------------------------------------
// cut / merged control volumes: one 256-thread block each
// ---------------------------------------------------------------------
// q: the control volume's slot in the instance's list of cut/merged volumes
__device__ inline void adj_cut_body(const Geo2D& G, const AdjBufs& B, const AdjParams& P, int part_base, int q,
                                    double* lds) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int m = G.irr[q];
  const int b0 = G.mptr[q];
  const int nm = min(G.mptr[q + 1] - b0, kMaxMembers);
  const int nx = G.nx, ny = G.ny, N = G.N, nvel = G.nvel;
  const double S = G.scv[m];
  const double rho = B.mom[4 * m], ux = B.mom[4 * m + 1], uy = B.mom[4 * m + 2], T = B.mom[4 * m + 3];
  const bool collide = P.kappa > 0.0;
  const double beta = collide ? P.dt * rho / P.kappa : 0.0;
  const double2* mu = B.mu_in + (size_t)m * nvel;
  const double2* xc = B.x + (size_t)m * nvel;
  const double Tw = P.t_wall;
  // reductions: relaxation, and per wall edge phi_w, d phi_w/dT_w, Lambda_k
  BgkSums A{0, 0, 0, 0, 0};
  double s[5] = {0, 0, 0, 0, 0};
  if (collide) {
    for (int p = tid; p < nvel; p += nth) {
      const double2 mm = mu[p], x = xc[p];
      bgk_terms(rho, ux, uy, T, vnd(P.vmin, P.dv, p % N), vnd(P.vmin, P.dv, p / N), S * mm.x, S * mm.y,
                x.x, x.y, s);
    }
    for (int k = 0; k < 5; ++k) s[k] = bsum(s[k], lds);
    A = chain(rho, ux, uy, T, s);
  }
  double den[kMaxMembers], lam[kMaxMembers];
  double pTw = 0.0;
  for (int t = 0; t < nm; ++t) {
    const int k = G.mem[b0 + t];
    den[t] = 0.0; lam[t] = 0.0;
    if (!(G.lw[k] > 0.0)) continue;
    double num = 0.0, dn = 0.0, dd = 0.0;
    for (int p = tid; p < nvel; p += nth) {
      const double vx = vnd(P.vmin, P.dv, p % N), vy = vnd(P.vmin, P.dv, p / N);
      const double cn = vx * G.nwx[k] + vy * G.nwy[k];
      if (cn > 0.0) num += cn * xc[p].x * P.w;
      else if (cn < 0.0) {
        const double Mw = maxw(1.0, 0.0, 0.0, Tw, vx, vy);
        dn += cn * Mw * P.w;
        dd += cn * Mw * ((vx * vx + vy * vy) / (2.0 * Tw * Tw) - 1.0 / Tw) * P.w;
      }
    }
    num = bsum(num, lds); dn = bsum(dn, lds); dd = bsum(dd, lds);
    const double phi = dn != 0.0 ? -num / dn : 0.0;
    const double dphi = dn != 0.0 ? num / (dn * dn) * dd : 0.0;
    double L = 0.0, dT = 0.0;
    for (int p = tid; p < nvel; p += nth) {
      const double vx = vnd(P.vmin, P.dv, p % N), vy = vnd(P.vmin, P.dv, p / N);
      const double cn = vx * G.nwx[k] + vy * G.nwy[k];
      if (cn >= 0.0) continue;
      const double Mw = maxw(1.0, 0.0, 0.0, Tw, vx, vy);
      const double dMw = Mw * ((vx * vx + vy * vy) / (2.0 * Tw * Tw) - 1.0 / Tw);
      const double2 mm = mu[p];
      const double lf = S * mm.x, lg = S * mm.y;
      L += cn * Mw * (lf + 0.5 * Tw * lg);
      const double dfw = dphi * Mw + phi * dMw;
      const double dgw = dphi * 0.5 * Tw * Mw + phi * (0.5 * Mw + 0.5 * Tw * dMw);
      dT += cn * (lf * dfw + lg * dgw);
    }
    L = bsum(L, lds);
    dT = bsum(dT, lds);
    den[t] = dn;
    lam[t] = L;
    pTw += -P.dt / S * G.lw[k] * dT;
  }
  double pux = 0.0, puy = 0.0;
  for (int p = tid; p < nvel; p += nth) {
    const double vx = vnd(P.vmin, P.dv, p % N), vy = vnd(P.vmin, P.dv, p / N);
    const double2 mm = mu[p];
    const double lf = S * mm.x, lg = S * mm.y;
    double of = (1.0 - beta) * lf, og = (1.0 - beta) * lg;
    if (collide) {
      of += beta * P.w * (A.Ar + A.Apx * vx + A.Apy * vy + A.Ae * 0.5 * (vx * vx + vy * vy)) +
            P.dt * P.w / P.kappa * A.C;
      og += beta * P.w * A.Ae;
    }
    for (int t = 0; t < nm; ++t) {
      const int k = G.mem[b0 + t];
      const int i = k % nx, j = k / nx;
      const double Le[4] = {G.lxp[k], G.lxm[k], G.lyp[k], G.lym[k]};
      const int nb[4] = {i + 1 < nx ? k + 1 : -1, i > 0 ? k - 1 : -1, j + 1 < ny ? k + nx : -1,
                         j > 0 ? k - nx : -1};
      const double cf[4] = {vx, -vx, vy, -vy};   // outward normal velocity of each edge
      for (int e = 0; e < 4; ++e) {
        if (Le[e] == 0.0) continue;
        if (nb[e] >= 0 && G.master[nb[e]] == m) continue;   // inside the control volume
        const double c = cf[e], cp = fmax(c, 0.0), cm = fmin(c, 0.0);
        of -= P.dt / S * Le[e] * cp * lf;
        og -= P.dt / S * Le[e] * cp * lg;
        if (nb[e] >= 0) {
          const double2 mn = B.mu_in[(size_t)nb[e] * nvel + p];
          of += P.dt * Le[e] * cp * mn.x;
          og += P.dt * Le[e] * cp * mn.y;
        } else if (cm != 0.0) {
          const double M = maxw(P.rho_in, P.ux_in, P.uy_in, P.t_in, vx, vy);
          const double tt = -P.dt / S * Le[e] * cm * (lf + 0.5 * P.t_in * lg) * M / P.t_in;
          pux += tt * (vx - P.ux_in);
          puy += tt * (vy - P.uy_in);
        }
      }
      const double Lw = G.lw[k];
      if (Lw > 0.0) {
        const double cn = vx * G.nwx[k] + vy * G.nwy[k];
        if (cn > 0.0) {
          of += -P.dt / S * Lw * cn * lf + P.dt / S * Lw * lam[t] * cn * P.w / den[t];
          og += -P.dt / S * Lw * cn * lg;
        }
      }
    }
    for (int t = 0; t < nm; ++t)
      B.mu_out[(size_t)G.mem[b0 + t] * nvel + p] = make_double2(of / S, og / S);
  }
  pux = bsum(pux, lds);
  puy = bsum(puy, lds);
  if (tid == 0) {
    double* pt = B.part + 4 * (size_t)(part_base + q);
    pt[0] += pTw;
    pt[1] += collide ? A.C * (-beta / P.kn) : 0.0;
    pt[2] += pux;
    pt[3] += puy;
  }
}

__global__ void __launch_bounds__(256) k_adj_cut2d(Geo2D G, AdjBufs B, AdjParams P, int part_base) {
  __shared__ double lds[8];
  adj_cut_body(G, B, P, part_base, blockIdx.x, lds);
}

// objective (drag or torque of the final state): mu^N at the members of every
// control volume with wall edges, and dJ/dT_w
__global__ void __launch_bounds__(256) k_adj_objective2d(Geo2D G, AdjBufs B, AdjParams P,
                                                         int part_base) {
  __shared__ double lds[8];
  const int q = blockIdx.x, tid = threadIdx.x, nth = blockDim.x;
  const int m = G.irr[q];
  const int b0 = G.mptr[q];
  const int nm = min(G.mptr[q + 1] - b0, kMaxMembers);
  const int N = G.N, nvel = G.nvel;
  const double S = G.scv[m];
  const double Tw = P.t_wall;
  const double2* xc = B.x + (size_t)m * nvel;
  double den[kMaxMembers], sin_[kMaxMembers], al[kMaxMembers], ga[kMaxMembers];
  double pTw = 0.0;
  for (int t = 0; t < nm; ++t) {
    const int k = G.mem[b0 + t];
    den[t] = 0.0; sin_[t] = 0.0; al[t] = 1.0; ga[t] = 0.0;
    if (!(G.lw[k] > 0.0)) continue;
    if (P.objective == 1) { al[t] = -(G.rwy[k] - B.body[1]); ga[t] = G.rwx[k] - B.body[0]; }
    double num = 0.0, dn = 0.0, dd = 0.0;
    for (int p = tid; p < nvel; p += nth) {
      const double vx = vnd(P.vmin, P.dv, p % N), vy = vnd(P.vmin, P.dv, p / N);
      const double cn = vx * G.nwx[k] + vy * G.nwy[k];
      if (cn > 0.0) num += cn * xc[p].x * P.w;
      else if (cn < 0.0) {
        const double Mw = maxw(1.0, 0.0, 0.0, Tw, vx, vy);
        dn += cn * Mw * P.w;
        dd += cn * Mw * ((vx * vx + vy * vy) / (2.0 * Tw * Tw) - 1.0 / Tw) * P.w;
      }
    }
    num = bsum(num, lds); dn = bsum(dn, lds); dd = bsum(dd, lds);
    const double phi = dn != 0.0 ? -num / dn : 0.0;
    const double dphi = dn != 0.0 ? num / (dn * dn) * dd : 0.0;
    double si = 0.0, sdT = 0.0;
    for (int p = tid; p < nvel; p += nth) {
      const double vx = vnd(P.vmin, P.dv, p % N), vy = vnd(P.vmin, P.dv, p / N);
      const double cn = vx * G.nwx[k] + vy * G.nwy[k];
      if (cn >= 0.0) continue;
      const double psi = al[t] * vx + ga[t] * vy;
      const double Mw = maxw(1.0, 0.0, 0.0, Tw, vx, vy);
      const double dMw = Mw * ((vx * vx + vy * vy) / (2.0 * Tw * Tw) - 1.0 / Tw);
      si += psi * cn * Mw * P.w;
      sdT += psi * cn * (dphi * Mw + phi * dMw) * P.w;
    }
    si = bsum(si, lds);
    sdT = bsum(sdT, lds);
    den[t] = dn;
    sin_[t] = si;
    pTw += G.lw[k] * sdT;
  }
  for (int p = tid; p < nvel; p += nth) {
    const double vx = vnd(P.vmin, P.dv, p % N), vy = vnd(P.vmin, P.dv, p / N);
    double of = 0.0;
    for (int t = 0; t < nm; ++t) {
      const int k = G.mem[b0 + t];
      if (!(G.lw[k] > 0.0)) continue;
      const double cn = vx * G.nwx[k] + vy * G.nwy[k];
      if (cn <= 0.0) continue;
      const double psi = al[t] * vx + ga[t] * vy;
      of += G.lw[k] * (psi * cn * P.w + sin_[t] * (-cn * P.w / den[t]));
    }
    for (int t = 0; t < nm; ++t)
      B.mu_out[(size_t)G.mem[b0 + t] * nvel + p] = make_double2(of / S, 0.0);
  }
  if (tid == 0) B.part[4 * (size_t)(part_base + q)] += pTw;
}

// initial state (inflow Maxwellian in every cell): sum_m S_m mu^0_m . dM/du
__global__ void __launch_bounds__(256) k_adj_initial2d(Geo2D G, AdjBufs B, AdjParams P, int part_base) {
  __shared__ double lds[8];
  const int c = blockIdx.x;
  const int m = G.master[c];
  if (m != c) return;                      // uniform over the block
  const int N = G.N, nvel = G.nvel;
  const double S = G.scv[m];
  const double2* mu = B.mu_in + (size_t)m * nvel;
  double pux = 0.0, puy = 0.0;
  for (int p = threadIdx.x; p < nvel; p += blockDim.x) {
    const double vx = vnd(P.vmin, P.dv, p % N), vy = vnd(P.vmin, P.dv, p / N);
    const double M = maxw(P.rho_in, P.ux_in, P.uy_in, P.t_in, vx, vy);
    const double t = S * (mu[p].x + 0.5 * P.t_in * mu[p].y) * M / P.t_in;
    pux += t * (vx - P.ux_in);
    puy += t * (vy - P.uy_in);
  }
  pux = bsum(pux, lds);
  puy = bsum(puy, lds);
  if (threadIdx.x == 0) {
    B.part[4 * (size_t)(part_base + c) + 2] += pux;
    B.part[4 * (size_t)(part_base + c) + 3] += puy;
  }
}

__global__ void k_fill0(double* __restrict__ p, size_t n) {
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
    p[t] = 0.0;
}

// fixed-order sum of the partial arrays into out[4], in two passes: block b
// of the first sums the partials [b*span, (b+1)*span) into mid[b] (kSumBlocks
// blocks), one block then sums mid in block order
constexpr int kSumBlocks = 256;

__global__ void __launch_bounds__(256) k_adj_sum(const double* __restrict__ part, int nparts, int span,
                                                 double* __restrict__ out) {
  __shared__ double lds[8];
  const int t0 = blockIdx.x * span, t1 = min(nparts, t0 + span);
  for (int r = 0; r < 4; ++r) {
    double s = 0.0;
    for (int t = t0 + threadIdx.x; t < t1; t += blockDim.x) s += part[4 * (size_t)t + r];
    s = bsum(s, lds);
    if (threadIdx.x == 0) out[4 * (size_t)blockIdx.x + r] = s;
  }
}

AdjParams adj_params(const cc_ctx* ctx, int objective) {
  AdjParams P;
  P.vmin = ctx->cfg.vmin;
  P.dv = ctx->dv;
  P.w = ctx->dv * ctx->dv;
  P.dt = ctx->dt;
  P.kappa = ctx->cfg.kn > 0.0 ? sqrt(M_PI) / 2.0 * ctx->cfg.kn * ctx->cfg.lref / sqrt(2.0) : 0.0;
  P.kn = ctx->cfg.kn;
  P.t_wall = ctx->body.t_wall;
  P.rho_in = ctx->cfg.inflow[0];
  P.ux_in = ctx->cfg.inflow[1];
  P.uy_in = ctx->cfg.inflow[2];
  P.t_in = ctx->cfg.inflow[4];
  P.objective = objective;
  return P;
}

}  // namespace

// Pool layout for the adjoint of nsteps steps with a checkpoint every K.
struct AdjLayout {
  size_t ckpt, ckmom, seg, segmom, mu0, mu1, part, mid, out, total;
  int nckpt, K, nparts, nreg_blocks;
};

static size_t al256(size_t x) { return (x + 255) / 256 * 256; }

static AdjLayout adj_layout(const cc_ctx* ctx, int nsteps, int K) {
  AdjLayout L;
  L.K = K;
  L.nckpt = (nsteps + K - 1) / K;
  const size_t st = ctx->state_bytes, mb = al256((size_t)ctx->ncell * 4 * sizeof(double));
  L.nreg_blocks = (ctx->ncell + 3) / 4;
  L.nparts = L.nreg_blocks + 2 * ctx->ncell + ctx->ncell;   // regular blocks, cut CVs, objective, initial
  size_t off = 0;
  L.ckpt = off; off += st * (size_t)L.nckpt;
  L.ckmom = off; off += mb * (size_t)L.nckpt;
  L.seg = off; off += st * (size_t)(K - 1);   // states 1 .. K-1 of a segment (state 0 is its checkpoint)
  L.segmom = off; off += mb * (size_t)K;
  L.mu0 = off; off += st;
  L.mu1 = off; off += st;
  L.part = off; off += al256((size_t)L.nparts * 4 * sizeof(double));
  L.mid = off; off += al256((size_t)kSumBlocks * 4 * sizeof(double));
  L.out = off; off += 256;
  L.total = off;
  return L;
}

size_t adjoint_workspace_bytes(const cc_ctx* ctx, int nsteps, int K) {
  return adj_layout(ctx, nsteps, K).total;
}

hipError_t launch_step_2d_ptrs(cc_ctx* ctx, const double2* in, double2* out, double* mom);
hipError_t launch_force_only_2d(cc_ctx* ctx, double* out4);

// Forward nsteps from the current state with checkpoints, objective of the
// final state, then the adjoint sweep segment by segment (restore, recompute
// the segment keeping every state and its moments, adjoint steps backwards).
// out (host) = J, dJ/dT_w, dJ/dKn, dJ/du_x, dJ/du_y.
hipError_t adjoint_run_2d(cc_ctx* ctx, int nsteps, int K, int objective, char* pool, double* out) {
  AdjLayout L = adj_layout(ctx, nsteps, K);
  hipStream_t s = ctx->stream;
  const size_t st = ctx->state_bytes;
  const size_t mb = al256((size_t)ctx->ncell * 4 * sizeof(double));
  AdjParams P = adj_params(ctx, objective);
  hipError_t e;
  double* part = (double*)(pool + L.part);
  k_fill0<<<512, 256, 0, s>>>(part, (size_t)L.nparts * 4);
  k_fill0<<<1024, 256, 0, s>>>((double*)(pool + L.mu0), st / 8);
  k_fill0<<<1024, 256, 0, s>>>((double*)(pool + L.mu1), st / 8);
  // forward with checkpoints: the state entering step n (n % K == 0) and the
  // moments it uses, so that the recomputation replays the forward bit for
  // bit.  The step before a checkpoint writes its output straight into the
  // checkpoint buffer (the context's output slot points there for that
  // step), and the next step reads it from there; only the first state is
  // copied.  The slots get their own buffers back on every exit.
  struct Slots {
    cc_ctx* c;
    void* own[2];
    ~Slots() { c->state[0] = own[0]; c->state[1] = own[1]; }
  } slots{ctx, {ctx->state[0], ctx->state[1]}};
  for (int n = 0; n < nsteps; ++n) {
    if (n == 0) {
      e = hipMemcpyAsync(pool + L.ckpt, ctx->state[ctx->cur], st, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return e;
    }
    if (n % K == 0) {
      e = hipMemcpyAsync(pool + L.ckmom + mb * (size_t)(n / K), ctx->s.mom,
                         (size_t)ctx->ncell * 4 * sizeof(double), hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return e;
    }
    const int out = 1 - ctx->cur;
    ctx->state[out] = (n + 1) % K == 0 && n + 1 < nsteps ? pool + L.ckpt + st * (size_t)((n + 1) / K)
                                                        : slots.own[out];
    e = launch_step_2d_fused(ctx, false, nullptr, nullptr, false);
    if (e != hipSuccess) return e;
  }
  // the final state (written to its own slot) is the current one
  ctx->state[1 - ctx->cur] = slots.own[1 - ctx->cur];
  // objective value and its sensitivity mu^N
  double* dev_out = (double*)(pool + L.out);
  e = launch_force_only_2d(ctx, dev_out);
  if (e != hipSuccess) return e;
  AdjBufs B;
  B.body = ctx->s.body;
  B.part = part;
  B.x = (const double2*)ctx->state[ctx->cur];
  B.mom = ctx->s.mom;
  B.mu_in = nullptr;
  B.mu_out = (double2*)(pool + L.mu0);
  const int cut_base = L.nreg_blocks, obj_base = L.nreg_blocks + ctx->ncell;
  if (ctx->n_irr > 0) k_adj_objective2d<<<ctx->n_irr, 256, 0, s>>>(ctx->g2, B, P, obj_base);
  int cur_mu = 0;   // mu^{n+1} lives in mu[cur_mu]
  char* mu[2] = {pool + L.mu0, pool + L.mu1};
  double* host_j = out;
  // backward over the segments
  for (int sg = L.nckpt - 1; sg >= 0; --sg) {
    const int n0 = sg * K, n1 = nsteps < n0 + K ? nsteps : n0 + K, len = n1 - n0;
    // state i of the segment: its checkpoint for i = 0 (read in place, never
    // written), else slot i-1 of the segment buffer
    auto state = [&](int i) { return i == 0 ? pool + L.ckpt + st * (size_t)sg : pool + L.seg + st * (size_t)(i - 1); };
    char* segmom = pool + L.segmom;
    e = hipMemcpyAsync(segmom, pool + L.ckmom + mb * (size_t)sg, (size_t)ctx->ncell * 4 * sizeof(double),
                       hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    for (int i = 0; i + 1 < len; ++i) {
      e = hipMemcpyAsync(segmom + mb * (i + 1), segmom + mb * i, (size_t)ctx->ncell * 4 * sizeof(double),
                         hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return e;
      e = launch_step_2d_ptrs(ctx, (const double2*)state(i), (double2*)state(i + 1),
                              (double*)(segmom + mb * (i + 1)));
      if (e != hipSuccess) return e;
    }
    for (int i = len - 1; i >= 0; --i) {
      B.x = (const double2*)state(i);
      B.mom = (const double*)(segmom + mb * i);
      B.mu_in = (const double2*)mu[cur_mu];
      B.mu_out = (double2*)mu[1 - cur_mu];
      // cut control volumes and regular cells write disjoint cells and
      // partial slots: the former run on the side stream beside the latter
      // (one after the other while profiling)
      const bool overlap = ctx->n_irr > 0 && ctx->side && !ctx->prof.on;
      if (overlap) {
        e = hipEventRecord(ctx->fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(ctx->side, ctx->fork, 0);
        if (e != hipSuccess) return e;
        k_adj_cut2d<<<ctx->n_irr, 256, 0, ctx->side>>>(ctx->g2, B, P, cut_base);
        e = hipEventRecord(ctx->join, ctx->side);
        if (e != hipSuccess) return e;
      } else if (ctx->n_irr > 0) {
        prof_begin(ctx, 1);
        k_adj_cut2d<<<ctx->n_irr, 256, 0, s>>>(ctx->g2, B, P, cut_base);
        prof_end(ctx, 1);
      }
      prof_begin(ctx, 0);
      k_adj_regular2d<<<L.nreg_blocks, 256, 0, s>>>(ctx->g2, B, P);
      prof_end(ctx, 0);
      if (overlap) {
        e = hipStreamWaitEvent(s, ctx->join, 0);
        if (e != hipSuccess) return e;
      }
      cur_mu = 1 - cur_mu;
    }
  }
  B.mu_in = (const double2*)mu[cur_mu];
  k_adj_initial2d<<<ctx->ncell, 256, 0, s>>>(ctx->g2, B, P, L.nreg_blocks + 2 * ctx->ncell);
  double* mid = (double*)(pool + L.mid);
  const int span = (L.nparts + kSumBlocks - 1) / kSumBlocks;
  k_adj_sum<<<kSumBlocks, 256, 0, s>>>(part, L.nparts, span, mid);
  k_adj_sum<<<1, 256, 0, s>>>(mid, kSumBlocks, kSumBlocks, dev_out + 4);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  double h[8];
  e = hipMemcpyAsync(h, dev_out, 8 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  host_j[0] = objective == 0 ? h[0] : h[2];
  host_j[1] = h[4];
  host_j[2] = h[5];
  host_j[3] = h[6];
  host_j[4] = h[7];
  return hipSuccess;
}

// ---------------------------------------------------------------------
// Batched adjoint: the instances of a batch run the same sequence as
// adjoint_run_2d in lock step (they share nsteps and K, hence the segment
// structure), each on its own pool, and every step of every phase is one
// launch over all instances: the forward steps (with checkpoints) and the
// segment recomputations through the batched step kernels with per-step
// descriptor tables, the adjoint steps through k_batch_adj_regular2d /
// k_batch_adj_cut2d with per-step buffer tables, the checkpoint and moment
// copies through one copy kernel.  Each instance's partial sums land in its
// own slots in the same order as alone, so its gradient is the same bit for
// bit as cc_adjoint's.  All tables are built on the host and uploaded once.
// ---------------------------------------------------------------------
namespace {

struct AdjInst {
  Geo2D G;
  AdjParams P;
  int cut_base;
};

// An item is a run of up to kAdjRun consecutive regular blocks (4 cells
// each) of one instance, so that the instance's descriptor is loaded once
// per run rather than once per 4 cells.
constexpr int kAdjRun = 8;

__global__ void __launch_bounds__(256) k_batch_adj_regular2d(const AdjInst* __restrict__ I,
                                                             const AdjBufs* __restrict__ Bs,
                                                             const int2* __restrict__ items, int n, int npad) {
  __shared__ double lds[4][4];
  // items in launch order: consecutive blocks go to different XCDs, as in
  // the single-instance kernel (mapping each XCD a contiguous range of the
  // list, as the forward tiles do, ran 10 % slower here)
  (void)npad;
  const int w = blockIdx.x;
  if (w >= n) return;
  const int2 it = items[w];
  const int inst = __builtin_amdgcn_readfirstlane(it.x);
  const int blk0 = __builtin_amdgcn_readfirstlane(it.y);
  const Geo2D G = I[inst].G;
  const AdjParams P = I[inst].P;
  const AdjBufs B = Bs[inst];
  const int nblk = (G.ncell + 3) / 4;
  const int end = min(blk0 + kAdjRun, nblk);
  for (int blk = blk0; blk < end; ++blk) adj_regular_body(G, B, P, blk, lds);
}

__global__ void __launch_bounds__(256) k_batch_adj_cut2d(const AdjInst* __restrict__ I,
                                                         const AdjBufs* __restrict__ Bs,
                                                         const int2* __restrict__ items, int n) {
  __shared__ double lds[8];
  if ((int)blockIdx.x >= n) return;
  const int2 it = items[blockIdx.x];
  const int inst = __builtin_amdgcn_readfirstlane(it.x);
  const int q = __builtin_amdgcn_readfirstlane(it.y);
  adj_cut_body(I[inst].G, Bs[inst], I[inst].P, I[inst].cut_base, q, lds);
}

struct CopyItem {
  const double* src;
  double* dst;
  size_t n;
};

// copy list blockIdx.y: src -> dst, n doubles
__global__ void k_copy_items(const CopyItem* __restrict__ items) {
  const CopyItem c = items[blockIdx.y];
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < c.n; t += (size_t)gridDim.x * blockDim.x)
    c.dst[t] = c.src[t];
}

struct BatchAdjPlan {
  std::vector<AdjLayout> L;
  std::vector<size_t> pool;          // offset of each instance's pool in the workspace
  size_t inst, bufs, fwd, copies, adj_items, cut_items, total;
  int nfwd, nbufs, ncopies, nadj_items, ncut_items;
};

BatchAdjPlan batch_adj_plan(const cc_batch* B, int nsteps, int K) {
  BatchAdjPlan X;
  const int n = (int)B->ctx.size();
  size_t off = 0;
  X.nadj_items = 0;
  X.ncut_items = 0;
  for (cc_ctx* c : B->ctx) {
    X.L.push_back(adj_layout(c, nsteps, K));
    X.pool.push_back(off);
    off += al256(X.L.back().total);
    X.nadj_items += (X.L.back().nreg_blocks + kAdjRun - 1) / kAdjRun;
    X.ncut_items += c->n_irr;
  }
  const int nckpt = (nsteps + K - 1) / K;
  X.nfwd = nsteps + (nsteps - nckpt);       // forward steps, then the segment recomputations
  X.nbufs = nsteps;                         // adjoint steps
  X.ncopies = 1 + 2 * nckpt + (nsteps - nckpt);
  X.inst = off; off += al256(n * sizeof(AdjInst));
  X.bufs = off; off += al256((size_t)X.nbufs * n * sizeof(AdjBufs));
  X.fwd = off; off += al256((size_t)X.nfwd * n * batch_desc_bytes());
  X.copies = off; off += al256((size_t)X.ncopies * n * sizeof(CopyItem));
  X.adj_items = off; off += al256((size_t)(X.nadj_items + 8) * sizeof(int2));
  X.cut_items = off; off += al256((size_t)(X.ncut_items + 1) * sizeof(int2));
  X.total = off;
  return X;
}

}  // namespace

size_t batch_adjoint_workspace_bytes(const cc_batch* B, int nsteps, int K) {
  return batch_adj_plan(B, nsteps, K).total;
}

// out (host, 5 per instance) = J, dJ/dT_w, dJ/dKn, dJ/du_x, dJ/du_y
hipError_t batch_adjoint_run_2d(cc_batch* Bt, int nsteps, int K, int objective, char* ws, double* out) {
  const int n = (int)Bt->ctx.size();
  const BatchAdjPlan X = batch_adj_plan(Bt, nsteps, K);
  hipStream_t s = Bt->stream;
  hipError_t e;
  const size_t dsz = batch_desc_bytes();
  // descriptor images of every instance (their tile and cut lists are
  // uploaded again, for the group tile heights in force now)
  std::vector<char> d0, d1;
  std::vector<int2> tiles, cuts;
  batch_fill(Bt, d0, d1, tiles, cuts);
  if (tiles.size() > Bt->tile_cap || cuts.size() > Bt->cut_cap) return hipErrorInvalidValue;
  Bt->ncut = (int)cuts.size();
  if (!tiles.empty() && (e = hipMemcpyAsync(Bt->d_tiles, tiles.data(), tiles.size() * sizeof(int2),
                                            hipMemcpyHostToDevice, s)) != hipSuccess)
    return e;
  if (!cuts.empty() && (e = hipMemcpyAsync(Bt->d_cuts, cuts.data(), cuts.size() * sizeof(int2),
                                           hipMemcpyHostToDevice, s)) != hipSuccess)
    return e;

  // ---- host tables
  std::vector<char> tab(X.total - X.inst, 0);
  auto at = [&](size_t off) { return tab.data() + (off - X.inst); };
  std::vector<int2> adj_items, cut_items;
  std::vector<char*> pool(n);
  std::vector<AdjParams> P(n);
  for (int i = 0; i < n; ++i) {
    cc_ctx* c = Bt->ctx[i];
    pool[i] = ws + X.pool[i];
    P[i] = adj_params(c, objective);
    AdjInst a;
    a.G = c->g2;
    a.P = P[i];
    a.cut_base = X.L[i].nreg_blocks;
    memcpy(at(X.inst) + i * sizeof(AdjInst), &a, sizeof(a));
    for (int b = 0; b < X.L[i].nreg_blocks; b += kAdjRun) adj_items.push_back(make_int2(i, b));
    for (int q = 0; q < c->n_irr; ++q) cut_items.push_back(make_int2(i, q));
  }
  memcpy(at(X.adj_items), adj_items.data(), adj_items.size() * sizeof(int2));
  memcpy(at(X.cut_items), cut_items.data(), cut_items.size() * sizeof(int2));
  const int nadj_pad = (X.nadj_items + 7) / 8 * 8;

  // the control flow of adjoint_run_2d, recorded as a list of operations
  enum { OP_COPY, OP_FWD, OP_ADJ };
  struct Op { int kind, idx; };
  std::vector<Op> ops;
  int nf = 0, nb = 0, nc = 0;
  auto add_copy = [&](auto&& item_of) {
    CopyItem* list = (CopyItem*)(at(X.copies)) + (size_t)nc * n;
    for (int i = 0; i < n; ++i) list[i] = item_of(i);
    ops.push_back({OP_COPY, nc++});
  };
  auto add_fwd = [&](auto&& ptrs_of) {
    char* set = at(X.fwd) + (size_t)nf * n * dsz;
    for (int i = 0; i < n; ++i) {
      memcpy(set + i * dsz, d0.data() + i * dsz, dsz);
      const double2* in;
      double2* o;
      double* mom;
      ptrs_of(i, in, o, mom);
      batch_desc_patch(set + i * dsz, in, o, mom);
    }
    ops.push_back({OP_FWD, nf++});
  };
  std::vector<size_t> st(n), mb(n);
  std::vector<int> cur(n);
  std::vector<char*> own0(n), own1(n), where(n);
  for (int i = 0; i < n; ++i) {
    cc_ctx* c = Bt->ctx[i];
    st[i] = c->state_bytes;
    mb[i] = al256((size_t)c->ncell * 4 * sizeof(double));
    cur[i] = c->cur;
    own0[i] = (char*)c->state[0];
    own1[i] = (char*)c->state[1];
    where[i] = (char*)c->state[c->cur];
  }
  auto own = [&](int i, int k) { return k ? own1[i] : own0[i]; };
  // forward with checkpoints
  for (int step = 0; step < nsteps; ++step) {
    if (step == 0)
      add_copy([&](int i) {
        return CopyItem{(const double*)where[i], (double*)(pool[i] + X.L[i].ckpt), st[i] / 8};
      });
    if (step % K == 0)
      add_copy([&](int i) {
        cc_ctx* c = Bt->ctx[i];
        return CopyItem{c->s.mom, (double*)(pool[i] + X.L[i].ckmom + mb[i] * (size_t)(step / K)),
                        (size_t)c->ncell * 4};
      });
    add_fwd([&](int i, const double2*& in, double2*& o, double*& mom) {
      const int outk = 1 - cur[i];
      char* dst = (step + 1) % K == 0 && step + 1 < nsteps ? pool[i] + X.L[i].ckpt + st[i] * (size_t)((step + 1) / K)
                                                           : own(i, outk);
      in = (const double2*)where[i];
      o = (double2*)dst;
      mom = Bt->ctx[i]->s.mom;
      cur[i] = outk;
      where[i] = dst;
    });
  }
  // backward over the segments
  const int nckpt = (nsteps + K - 1) / K;
  int cur_mu = 0;
  std::vector<int> bw_order;
  for (int sg = nckpt - 1; sg >= 0; --sg) {
    const int n0 = sg * K, n1 = nsteps < n0 + K ? nsteps : n0 + K, len = n1 - n0;
    auto state = [&](int i, int k) -> char* {
      return k == 0 ? pool[i] + X.L[i].ckpt + st[i] * (size_t)sg : pool[i] + X.L[i].seg + st[i] * (size_t)(k - 1);
    };
    add_copy([&](int i) {
      return CopyItem{(const double*)(pool[i] + X.L[i].ckmom + mb[i] * (size_t)sg),
                      (double*)(pool[i] + X.L[i].segmom), (size_t)Bt->ctx[i]->ncell * 4};
    });
    for (int k = 0; k + 1 < len; ++k) {
      add_copy([&](int i) {
        char* sm = pool[i] + X.L[i].segmom;
        return CopyItem{(const double*)(sm + mb[i] * k), (double*)(sm + mb[i] * (k + 1)),
                        (size_t)Bt->ctx[i]->ncell * 4};
      });
      add_fwd([&](int i, const double2*& in, double2*& o, double*& mom) {
        in = (const double2*)state(i, k);
        o = (double2*)state(i, k + 1);
        mom = (double*)(pool[i] + X.L[i].segmom + mb[i] * (k + 1));
      });
    }
    for (int k = len - 1; k >= 0; --k) {
      AdjBufs* set = (AdjBufs*)(at(X.bufs)) + (size_t)nb * n;
      for (int i = 0; i < n; ++i) {
        char* mu[2] = {pool[i] + X.L[i].mu0, pool[i] + X.L[i].mu1};
        AdjBufs b;
        b.x = (const double2*)state(i, k);
        b.mom = (const double*)(pool[i] + X.L[i].segmom + mb[i] * k);
        b.mu_in = (const double2*)mu[cur_mu];
        b.mu_out = (double2*)mu[1 - cur_mu];
        b.part = (double*)(pool[i] + X.L[i].part);
        b.body = Bt->ctx[i]->s.body;
        set[i] = b;
      }
      ops.push_back({OP_ADJ, nb++});
      cur_mu = 1 - cur_mu;
    }
  }
  if (nf != X.nfwd || nb != X.nbufs || nc != X.ncopies) return hipErrorInvalidValue;
  e = hipMemcpyAsync(ws + X.inst, tab.data(), tab.size(), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;

  // ---- device work
  for (int i = 0; i < n; ++i) {
    const AdjLayout& L = X.L[i];
    k_fill0<<<512, 256, 0, s>>>((double*)(pool[i] + L.part), (size_t)L.nparts * 4);
    k_fill0<<<1024, 256, 0, s>>>((double*)(pool[i] + L.mu0), st[i] / 8);
    k_fill0<<<1024, 256, 0, s>>>((double*)(pool[i] + L.mu1), st[i] / 8);
  }
  const AdjInst* dI = (const AdjInst*)(ws + X.inst);
  const int2* dadj = (const int2*)(ws + X.adj_items);
  const int2* dcut = (const int2*)(ws + X.cut_items);
  hipStream_t side[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t fork = nullptr, join = nullptr;
  struct Cleanup {
    hipStream_t* side;
    hipEvent_t* fork;
    hipEvent_t* join;
    ~Cleanup() {
      for (int k = 0; k < 4; ++k)
        if (side[k]) hipStreamDestroy(side[k]);
      if (*fork) hipEventDestroy(*fork);
      if (*join) hipEventDestroy(*join);
    }
  } cleanup{side, &fork, &join};
  for (int k = 0; k < 4; ++k)
    if ((e = hipStreamCreateWithFlags(&side[k], hipStreamNonBlocking)) != hipSuccess) return e;
  if ((e = hipEventCreateWithFlags(&fork, hipEventDisableTiming)) != hipSuccess) return e;
  if ((e = hipEventCreateWithFlags(&join, hipEventDisableTiming)) != hipSuccess) return e;
  auto run = [&](const Op& op) -> hipError_t {
    if (op.kind == OP_COPY) {
      k_copy_items<<<dim3(1024, n), 256, 0, s>>>((const CopyItem*)(ws + X.copies) + (size_t)op.idx * n);
    } else if (op.kind == OP_FWD) {
      return batch_launch_desc(Bt, ws + X.fwd + (size_t)op.idx * n * dsz, side, 4);
    } else {
      const AdjBufs* set = (const AdjBufs*)(ws + X.bufs) + (size_t)op.idx * n;
      // cut control volumes beside the regular cells (disjoint cells and slots)
      if (X.ncut_items > 0) {
        hipError_t r = hipEventRecord(fork, s);
        if (r == hipSuccess) r = hipStreamWaitEvent(side[0], fork, 0);
        if (r != hipSuccess) return r;
        k_batch_adj_cut2d<<<X.ncut_items, 256, 0, side[0]>>>(dI, set, dcut, X.ncut_items);
        if ((r = hipEventRecord(join, side[0])) != hipSuccess) return r;
      }
      k_batch_adj_regular2d<<<nadj_pad, 256, 0, s>>>(dI, set, dadj, X.nadj_items, nadj_pad);
      if (X.ncut_items > 0) return hipStreamWaitEvent(s, join, 0);
    }
    return hipGetLastError();
  };
  // forward phase: operations up to the first adjoint step's segment start
  // are recorded in order; the objective sits between the forward and the
  // backward operations
  size_t k = 0;
  const size_t nforward_ops = 1 + (size_t)nckpt + (size_t)nsteps;   // initial copy, moment copies, steps
  for (; k < nforward_ops; ++k)
    if ((e = run(ops[k])) != hipSuccess) return e;
  // instance state after the forward: the final state is current
  for (int i = 0; i < n; ++i) {
    cc_ctx* c = Bt->ctx[i];
    const int steps_parity = nsteps & 1;
    c->cur = cur[i];
    c->step_parity ^= steps_parity;
    (void)steps_parity;
  }
  std::vector<double> hout(8 * (size_t)n, 0.0);
  for (int i = 0; i < n; ++i) {
    cc_ctx* c = Bt->ctx[i];
    double* dev_out = (double*)(pool[i] + X.L[i].out);
    if ((e = launch_force_only_2d(c, dev_out)) != hipSuccess) return e;
    AdjBufs b;
    b.body = c->s.body;
    b.part = (double*)(pool[i] + X.L[i].part);
    b.x = (const double2*)c->state[c->cur];
    b.mom = c->s.mom;
    b.mu_in = nullptr;
    b.mu_out = (double2*)(pool[i] + X.L[i].mu0);
    if (c->n_irr > 0)
      k_adj_objective2d<<<c->n_irr, 256, 0, s>>>(c->g2, b, P[i], X.L[i].nreg_blocks + c->ncell);
  }
  for (; k < ops.size(); ++k)
    if ((e = run(ops[k])) != hipSuccess) return e;
  for (int i = 0; i < n; ++i) {
    cc_ctx* c = Bt->ctx[i];
    const AdjLayout& L = X.L[i];
    AdjBufs b;
    b.body = c->s.body;
    b.part = (double*)(pool[i] + L.part);
    b.x = nullptr;
    b.mom = nullptr;
    b.mu_in = (const double2*)(cur_mu ? pool[i] + L.mu1 : pool[i] + L.mu0);
    b.mu_out = nullptr;
    k_adj_initial2d<<<c->ncell, 256, 0, s>>>(c->g2, b, P[i], L.nreg_blocks + 2 * c->ncell);
    double* mid = (double*)(pool[i] + L.mid);
    double* dev_out = (double*)(pool[i] + L.out);
    const int span = (L.nparts + kSumBlocks - 1) / kSumBlocks;
    k_adj_sum<<<kSumBlocks, 256, 0, s>>>(b.part, L.nparts, span, mid);
    k_adj_sum<<<1, 256, 0, s>>>(mid, kSumBlocks, kSumBlocks, dev_out + 4);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(hout.data() + 8 * (size_t)i, dev_out, 8 * sizeof(double), hipMemcpyDeviceToHost,
                            s)) != hipSuccess)
      return e;
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  for (int i = 0; i < n; ++i) {
    const double* h = hout.data() + 8 * (size_t)i;
    out[5 * i + 0] = objective == 0 ? h[0] : h[2];
    out[5 * i + 1] = h[4];
    out[5 * i + 2] = h[5];
    out[5 * i + 3] = h[6];
    out[5 * i + 4] = h[7];
  }
  return hipSuccess;
}

}  // namespace ccdvm
