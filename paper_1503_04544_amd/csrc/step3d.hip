// Device step of the 3D cut-cell scheme (Section 5.1, eq. eq-schema3D, fixed
// body) with the BGK relaxation (eq. MaxwellianTD, tau = (sqrt(pi)/2) Kn
// L_ref / (sqrt(2) rho)) and the diffuse wall of zero net mass flux.
//
// Layout: double state[c][p] = F, p = (p3*N + p2)*N + p1.
//
// Regular cells (gas, a control volume of one cell) are streamed by
// k_step3d.  The velocity set is cut into chunks with a fixed sign of v_y
// (half of the p2 range) and of v_z (G3 consecutive p3 of one half); a chunk
// holds G3*N*N/2 velocities, R per lane, and is contiguous per p3.  A block
// of 16 waves owns a 4 x 4 tile of x-pencils (j, k) for one chunk and marches
// along x: the x-upwind value comes from a register window (previous cell
// for v_x > 0, the prefetched next cell for v_x < 0); the y- and z-upwind
// cells of one chunk lie in a fixed direction, so each wave publishes its
// cell in LDS for the neighbouring pencils of the tile (one barrier per
// x-step) and only the waves on the upwind edge of the tile read the
// neighbouring tile's cell from memory.  Each wave reduces the chunk's
// contribution to the moments of the new value; k_mom3d sums the chunks
// before the next step.
//
// Cut cells and control volumes with merged members go to k_cut3d, one
// 256-thread block each.
#include <hip/hip_runtime.h>

#include <math.h>

#include "ccdvm_impl.h"

namespace ccdvm {
namespace {

constexpr int kWave = 64;
constexpr int kTY = 4, kTZ = 4, kTileWaves = kTY * kTZ;
constexpr int kPD3 = 2;   // cells prefetched ahead of the next one

__device__ inline double wave_sum3(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// sum over the 4 waves of a 256-thread block, added in wave order
__device__ inline double block_sum(double v, double* lds) {
  v = wave_sum3(v);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[wave] = v;
  __syncthreads();
  return ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

__device__ inline double vnode3(double vmin, double dv, int idx) { return vmin + (idx + 0.5) * dv; }

// Chunking of the velocity set for N nodes per axis (N even, symmetric box).
template <int N>
struct Chunk3 {
  static constexpr int H = N / 2;                 // p2 (or p3) values of one sign
  static constexpr int E1 = H * N;                // velocities of one (p3, half of p2)
  static constexpr int G3 = (H % 2 == 0) ? 2 : (H % 3 == 0 ? 3 : 1);  // p3 per chunk
  static constexpr int CH = G3 * E1;              // velocities per chunk
  static constexpr int R = (CH + kWave - 1) / kWave;
  static constexpr int NCH = 4 * H / G3;          // chunks
};

// offset within the cell of element e of chunk ch
template <int N>
__device__ inline int chunk_offset(int ch, int e) {
  using C = Chunk3<N>;
  const int sy = ch & 1, p3b = (ch >> 1) * C::G3;
  return (p3b + e / C::E1) * N * N + sy * C::E1 + e % C::E1;
}

struct Step3Args {
  const double* in;
  double* out;
  const int* kind;
  const double* mom;    // 8 per cell: A, ux, uy, uz, 1/(2T), dt/tau, rho, -
  double* part;         // per cell and chunk: sums of F, v F, |v|^2 F (5)
  const double* ghost;  // farfield values
  int nx, ny, nz, nvel;
  int ntj, ntiles, nblk, per;
  double vmin, dv, cxf, cyf, czf;   // dt/dx, dt/dy, dt/dz
};

template <int N>
__global__ void __launch_bounds__(1024) k_step3d(const Step3Args A) {
  using C = Chunk3<N>;
  constexpr int R = C::R;
  __shared__ double xch[2][kTileWaves][R][kWave];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // XCD-aware order: block b runs on XCD b % 8; the blocks of one XCD are
  // consecutive tiles of one chunk, so the neighbouring tiles whose edge
  // cells a tile reads are resident on the same L2
  const int b = blockIdx.x;
  const int logical = (b & 7) * A.per + (b >> 3);
  if (logical >= A.nblk) return;
  const int ch = logical / A.ntiles, tile = logical - ch * A.ntiles;
  const int ty = wave & 3, tz = wave >> 2;
  const int tj = tile % A.ntj, tk = tile / A.ntj;
  const int j = tj * kTY + ty, k = tk * kTZ + tz;
  const bool valid = j < A.ny && k < A.nz;
  const int sy = ch & 1, p3b = (ch >> 1) * C::G3;
  const int dyu = sy ? -1 : 1, dzu = p3b >= C::H ? -1 : 1;   // upwind direction
  const int jy = j + dyu, kz = k + dzu, tyu = ty + dyu, tzu = tz + dzu;
  const bool y_dom = jy >= 0 && jy < A.ny, z_dom = kz >= 0 && kz < A.nz;
  const bool y_lds = y_dom && tyu >= 0 && tyu < kTY;
  const bool z_lds = z_dom && tzu >= 0 && tzu < kTZ;
  const int wy = y_lds ? tz * kTY + tyu : 0, wz = z_lds ? tzu * kTY + ty : 0;
  const int nx = A.nx, nvel = A.nvel;
  const size_t pencil = (size_t)(k * A.ny + j) * nx;
  const double* __restrict__ own_base = A.in + pencil * nvel;
  // halo rows: the neighbouring tile's pencil, or the farfield outside
  const double* __restrict__ y_base =
      y_dom ? A.in + (size_t)(k * A.ny + jy) * nx * nvel : A.ghost;
  const double* __restrict__ z_base =
      z_dom ? A.in + (size_t)(kz * A.ny + j) * nx * nvel : A.ghost;
  const size_t y_step = y_dom ? nvel : 0, z_step = z_dom ? nvel : 0;
  const bool y_glob = valid && !y_lds, z_glob = valid && !z_lds;

  // Per-lane velocity indices are recomputed where they are used from a
  // laundered copy of the lane id, so that the compiler does not keep R sets
  // of velocity constants live across the x loop.
  auto offset = [&](int lv, int r) { return chunk_offset<N>(ch, min(r * kWave + lv, C::CH - 1)); };
  auto active = [&](int lv, int r) { return valid && r * kWave + lv < C::CH; };
  auto load_row = [&](double (&dst)[R], const double* __restrict__ row, int lv) {
#pragma unroll
    for (int r = 0; r < R; ++r) dst[r] = active(lv, r) ? row[offset(lv, r)] : 0.0;
  };
  auto own_row = [&](int i) -> const double* {
    return i < nx ? own_base + (size_t)i * nvel : A.ghost;
  };
  double prv[R], cur[R], q[kPD3 + 1][R];
  load_row(prv, A.ghost, lane);
  load_row(cur, own_base, lane);
#pragma unroll
  for (int d = 0; d <= kPD3; ++d) {
    if (1 + d <= nx) load_row(q[d], own_row(1 + d), lane);
    else
#pragma unroll
      for (int r = 0; r < R; ++r) q[d][r] = 0.0;
  }
  const double vmin = A.vmin, dv = A.dv;
  for (int i = 0; i < nx; ++i) {
    int lv = lane;
    asm volatile("" : "+v"(lv));
    // prefetch: own cell i+kPD3+2 (the farfield past the end); the halo of
    // cell i is read now and waited for after the exchange barrier
    double qn[R], hy[R], hz[R];
    const int ia = i + kPD3 + 2;
    if (ia <= nx) load_row(qn, own_row(ia), lv);
    else
#pragma unroll
      for (int r = 0; r < R; ++r) qn[r] = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool a = active(lv, r);
      const int o = offset(lv, r);
      hy[r] = y_glob && a ? y_base[(size_t)i * y_step + o] : 0.0;
      hz[r] = z_glob && a ? z_base[(size_t)i * z_step + o] : 0.0;
    }
    const int s = i & 1;
#pragma unroll
    for (int r = 0; r < R; ++r) xch[s][wave][r][lv] = cur[r];
    __syncthreads();
    const int c = (int)(pencil + i);
    if (valid && A.kind[c] == KIND_REGULAR) {
      const double* mc = A.mom + 8 * (size_t)c;
      const double Am = mc[0], ux = mc[1], uy = mc[2], uz = mc[3], inv2T = mc[4], nu = mc[5];
      double tx = 0.0, tyy = 0.0, tzz = 0.0;
      if (lv < N) {
        const double v = vnode3(vmin, dv, lv);
        tx = exp(-(v - ux) * (v - ux) * inv2T);
        tyy = exp(-(v - uy) * (v - uy) * inv2T);
        tzz = exp(-(v - uz) * (v - uz) * inv2T);
      }
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
      double* orow = A.out + (pencil + i) * (size_t)nvel;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = min(r * kWave + lv, C::CH - 1);
        const int rem = e % C::E1;
        const int p1 = rem % N, p2 = sy * C::H + rem / N, p3 = p3b + e / C::E1;
        const double vx = vnode3(vmin, dv, p1), vy = vnode3(vmin, dv, p2), vz = vnode3(vmin, dv, p3);
        const double E = Am * __shfl(tx, p1, kWave) * __shfl(tyy, p2, kWave) * __shfl(tzz, p3, kWave);
        const double yv = y_lds ? xch[s][wy][r][lv] : hy[r];
        const double zv = z_lds ? xch[s][wz][r][lv] : hz[r];
        const double f = cur[r];
        const double fxu = p1 >= C::H ? prv[r] : q[0][r];
        const double fn = f - A.cxf * fabs(vx) * (f - fxu) - A.cyf * fabs(vy) * (f - yv) -
                          A.czf * fabs(vz) * (f - zv) + nu * (E - f);
        if (active(lv, r)) {
          __builtin_nontemporal_store(fn, &orow[offset(lv, r)]);
          s0 += fn; s1 += vx * fn; s2 += vy * fn; s3 += vz * fn;
          s4 += (vx * vx + vy * vy + vz * vz) * fn;
        }
      }
      s0 = wave_sum3(s0); s1 = wave_sum3(s1); s2 = wave_sum3(s2);
      s3 = wave_sum3(s3); s4 = wave_sum3(s4);
      if (lv == 0) {
        double* pp = A.part + ((size_t)c * C::NCH + ch) * 5;
        pp[0] = s0; pp[1] = s1; pp[2] = s2; pp[3] = s3; pp[4] = s4;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      prv[r] = cur[r];
      cur[r] = q[0][r];
#pragma unroll
      for (int d = 0; d < kPD3; ++d) q[d][r] = q[d + 1][r];
      q[kPD3][r] = qn[r];
    }
  }
}

// partial moments of the current state, per regular cell and chunk (one
// wave per cell)
template <int N>
__global__ void __launch_bounds__(256) k_part3d(Geo3D G, const double* __restrict__ in,
                                               double* __restrict__ part, double vmin, double dv) {
  using C = Chunk3<N>;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= G.ncell || G.kind[c] != KIND_REGULAR) return;
  const double* row = in + (size_t)c * G.nvel;
  for (int ch = 0; ch < C::NCH; ++ch) {
    const int sy = ch & 1, p3b = (ch >> 1) * C::G3;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
    for (int r = 0; r < C::R; ++r) {
      const int e = r * kWave + lane;
      if (e >= C::CH) continue;
      const int rem = e % C::E1;
      const double vx = vnode3(vmin, dv, rem % N), vy = vnode3(vmin, dv, sy * C::H + rem / N),
                   vz = vnode3(vmin, dv, p3b + e / C::E1);
      const double f = row[chunk_offset<N>(ch, e)];
      s0 += f; s1 += vx * f; s2 += vy * f; s3 += vz * f;
      s4 += (vx * vx + vy * vy + vz * vz) * f;
    }
    s0 = wave_sum3(s0); s1 = wave_sum3(s1); s2 = wave_sum3(s2);
    s3 = wave_sum3(s3); s4 = wave_sum3(s4);
    if (lane == 0) {
      double* pp = part + ((size_t)c * C::NCH + ch) * 5;
      pp[0] = s0; pp[1] = s1; pp[2] = s2; pp[3] = s3; pp[4] = s4;
    }
  }
}

struct Mom3Params {
  double w, dt, tau_coef, vol;
  int nch;
};

// moments of the regular cells from the chunk sums (eq. MacroscopicTD):
// rho, u, T = (2E/rho - |u|^2)/3, and the BGK coefficients; block partials
// of the mass sum_c V_c rho_c
__global__ void __launch_bounds__(256) k_mom3d(Geo3D G, const double* __restrict__ part,
                                              double* __restrict__ mom, double* __restrict__ mpart,
                                              Mom3Params P) {
  __shared__ double lds[4];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double ms = 0.0;
  if (c < G.ncell && G.kind[c] == KIND_REGULAR) {
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const double* pp = part + (size_t)c * P.nch * 5;
    for (int ch = 0; ch < P.nch; ++ch)
      for (int q = 0; q < 5; ++q) s[q] += pp[5 * ch + q];
    const double rho = s[0] * P.w;
    const double ux = s[1] * P.w / rho, uy = s[2] * P.w / rho, uz = s[3] * P.w / rho;
    const double en = 0.5 * s[4] * P.w;
    const double T = (2.0 * en / rho - (ux * ux + uy * uy + uz * uz)) / 3.0;
    double* mo = mom + 8 * (size_t)c;
    mo[0] = rho / pow(2.0 * M_PI * T, 1.5);
    mo[1] = ux; mo[2] = uy; mo[3] = uz;
    mo[4] = 0.5 / T;
    mo[5] = P.tau_coef > 0.0 ? P.dt * rho / P.tau_coef : 0.0;
    mo[6] = rho;
    ms = P.vol * rho;
  }
  ms = block_sum(ms, lds);
  if (threadIdx.x == 0) mpart[blockIdx.x] = ms;
}

struct Cut3Params {
  double vmin, dv, w, dt, tau_coef, t_wall;
  int write_state;
};

__device__ inline double maxw3(double rho, double ux, double uy, double uz, double T, double vx,
                               double vy, double vz) {
  const double ex = vx - ux, ey = vy - uy, ez = vz - uz;
  return rho / pow(2.0 * M_PI * T, 1.5) * exp(-(ex * ex + ey * ey + ez * ez) / (2.0 * T));
}

// One control volume that is cut or owns merged cells: wall density of each
// wall face (zero net mass flux, Section 5.1), fluxes through the six
// Cartesian faces and the wall face of every member, explicit update with
// relaxation, redistribution to the members; wall stress -> force and the
// mass of the state at t^n.  write_state == 0: force and mass only.
__global__ void __launch_bounds__(256) k_cut3d(Geo3D G, const double* __restrict__ in,
                                              double* __restrict__ out, double* __restrict__ fslot,
                                              double* __restrict__ mpart, Cut3Params P) {
  __shared__ double lds[4];
  const int tid = threadIdx.x, nth = blockDim.x;
  const int q = blockIdx.x;
  const int m = G.irr[q];
  const int b = G.mptr[q], nm = G.mptr[q + 1] - b;
  const int N = G.N, nvel = G.nvel, nx = G.nx, ny = G.ny, nz = G.nz;
  const double* own = in + (size_t)m * nvel;
  // moments of the control volume's value
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
  for (int p = tid; p < nvel; p += nth) {
    const double vx = vnode3(P.vmin, P.dv, p % N), vy = vnode3(P.vmin, P.dv, (p / N) % N),
                 vz = vnode3(P.vmin, P.dv, p / (N * N));
    const double f = own[p];
    s0 += f; s1 += vx * f; s2 += vy * f; s3 += vz * f;
    s4 += (vx * vx + vy * vy + vz * vz) * f;
  }
  s0 = block_sum(s0, lds); s1 = block_sum(s1, lds); s2 = block_sum(s2, lds);
  s3 = block_sum(s3, lds); s4 = block_sum(s4, lds);
  const double rho = s0 * P.w, ux = s1 * P.w / rho, uy = s2 * P.w / rho, uz = s3 * P.w / rho;
  const double T = (2.0 * (0.5 * s4 * P.w) / rho - (ux * ux + uy * uy + uz * uz)) / 3.0;
  const double nu = P.tau_coef > 0.0 ? P.dt * rho / P.tau_coef : 0.0;
  const double V = G.vcv[m];
  const double Tw = P.t_wall;
  double phiw[kMaxMembers];
  for (int t = 0; t < nm; ++t) {
    const int k = G.mem[b + t];
    phiw[t] = 0.0;
    if (!(G.aw[k] > 0.0)) continue;
    const double n0 = G.nwx[k], n1 = G.nwy[k], n2 = G.nwz[k];
    double num = 0.0, den = 0.0;
    for (int p = tid; p < nvel; p += nth) {
      const double vx = vnode3(P.vmin, P.dv, p % N), vy = vnode3(P.vmin, P.dv, (p / N) % N),
                   vz = vnode3(P.vmin, P.dv, p / (N * N));
      const double cn = vx * n0 + vy * n1 + vz * n2;
      if (cn > 0.0) num += cn * own[p];
      else if (cn < 0.0) den += cn * maxw3(1.0, 0.0, 0.0, 0.0, Tw, vx, vy, vz);
    }
    num = block_sum(num, lds);
    den = block_sum(den, lds);
    phiw[t] = den != 0.0 ? -num / den : 0.0;
  }
  double sx[kMaxMembers], sy[kMaxMembers], sz[kMaxMembers];
  for (int t = 0; t < kMaxMembers; ++t) { sx[t] = 0.0; sy[t] = 0.0; sz[t] = 0.0; }
  for (int p = tid; p < nvel; p += nth) {
    const double v[3] = {vnode3(P.vmin, P.dv, p % N), vnode3(P.vmin, P.dv, (p / N) % N),
                         vnode3(P.vmin, P.dv, p / (N * N))};
    const double fo = own[p];
    double Rs = 0.0;
    for (int t = 0; t < nm; ++t) {
      const int k = G.mem[b + t];
      const int i = k % nx, j = (k / nx) % ny, kk = k / (nx * ny);
      const double S[6] = {G.sxm[k], G.sxp[k], G.sym[k], G.syp[k], G.szm[k], G.szp[k]};
      const bool inside[6] = {i > 0, i + 1 < nx, j > 0, j + 1 < ny, kk > 0, kk + 1 < nz};
      const long long stride[3] = {1, nx, (long long)nx * ny};
      for (int f = 0; f < 6; ++f) {
        if (!(S[f] > 0.0)) continue;
        const int d = f >> 1;
        const double cvel = (f & 1) ? v[d] : -v[d];   // outward normal velocity
        const double fn = inside[f] ? in[(size_t)(k + ((f & 1) ? stride[d] : -stride[d])) * nvel + p]
                                    : G.ghost[p];
        Rs += S[f] * (fmax(cvel, 0.0) * fo + fmin(cvel, 0.0) * fn);
      }
      const double aw = G.aw[k];
      if (aw > 0.0) {
        const double cn = v[0] * G.nwx[k] + v[1] * G.nwy[k] + v[2] * G.nwz[k];
        const double fw = phiw[t] * maxw3(1.0, 0.0, 0.0, 0.0, Tw, v[0], v[1], v[2]);
        Rs += aw * (fmin(cn, 0.0) * fw + fmax(cn, 0.0) * fo);
        const double fv = cn < 0.0 ? fw : (cn > 0.0 ? fo : 0.0);
        sx[t] += v[0] * cn * fv;
        sy[t] += v[1] * cn * fv;
        sz[t] += v[2] * cn * fv;
      }
    }
    if (P.write_state) {
      const double E = nu != 0.0 ? maxw3(rho, ux, uy, uz, T, v[0], v[1], v[2]) : 0.0;
      const double fn = fo - P.dt / V * Rs + nu * (E - fo);
      for (int t = 0; t < nm; ++t) out[(size_t)G.mem[b + t] * nvel + p] = fn;
    }
  }
  double Fx = 0.0, Fy = 0.0, Fz = 0.0;
  for (int t = 0; t < nm; ++t) {
    const int k = G.mem[b + t];
    if (!(G.aw[k] > 0.0)) continue;
    const double ax = block_sum(sx[t], lds) * P.w, ay = block_sum(sy[t], lds) * P.w,
                 az = block_sum(sz[t], lds) * P.w;
    Fx += ax * G.aw[k];
    Fy += ay * G.aw[k];
    Fz += az * G.aw[k];
  }
  if (tid == 0) {
    fslot[3 * q + 0] = Fx;
    fslot[3 * q + 1] = Fy;
    fslot[3 * q + 2] = Fz;
    mpart[q] = V * rho;
  }
}

// diag row: force summed over the control volumes in list order, mass over
// the regular-cell block partials then the control volumes
__global__ void __launch_bounds__(256) k_reduce3d(const double* __restrict__ fslot, int ncv,
                                                 const double* __restrict__ mreg, int nreg,
                                                 const double* __restrict__ mcut,
                                                 double* __restrict__ row) {
  __shared__ double lds[4];
  double fx = 0.0, fy = 0.0, fz = 0.0, ms = 0.0, mc = 0.0;
  for (int t = threadIdx.x; t < ncv; t += blockDim.x) {
    fx += fslot[3 * t]; fy += fslot[3 * t + 1]; fz += fslot[3 * t + 2];
    mc += mcut[t];
  }
  for (int t = threadIdx.x; t < nreg; t += blockDim.x) ms += mreg[t];
  fx = block_sum(fx, lds); fy = block_sum(fy, lds); fz = block_sum(fz, lds);
  ms = block_sum(ms, lds); mc = block_sum(mc, lds);
  if (threadIdx.x == 0) {
    row[0] = fx; row[1] = fy; row[2] = fz;
    row[3] = ms + mc;
  }
}

// merge over the control volumes with more than one member (Section 5.1
// step 2): value = sum_k Vbar_k F_k / V, written to every member
__global__ void __launch_bounds__(256) k_merge3d(Geo3D G, double* __restrict__ st) {
  const int q = blockIdx.x;
  const int b = G.mptr[q], nm = G.mptr[q + 1] - b;
  if (nm <= 1) return;
  const int m = G.irr[q];
  const int nvel = G.nvel;
  for (int p = threadIdx.x; p < nvel; p += blockDim.x) {
    double acc = 0.0;
    for (int t = 0; t < nm; ++t) {
      const int k = G.mem[b + t];
      acc += G.vbar[k] * st[(size_t)k * nvel + p];
    }
    const double v = acc / G.vcv[m];
    for (int t = 0; t < nm; ++t) st[(size_t)G.mem[b + t] * nvel + p] = v;
  }
}

__global__ void k_init3d(Geo3D G, double* __restrict__ st) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)G.ncell * G.nvel) return;
  const int c = (int)(t / G.nvel), p = (int)(t % G.nvel);
  st[t] = G.kind[c] == KIND_SOLID ? 0.0 : G.ghost[p];
}

__global__ void k_load3d(Geo3D G, double* __restrict__ st, const double* __restrict__ f) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)G.ncell * G.nvel) return;
  const int c = (int)(t / G.nvel);
  st[t] = G.kind[c] == KIND_SOLID ? 0.0 : f[t];
}

// 14 moments per cell (eq. MacroscopicTD): rho, u, T, Sigma (xx, xy, xz, yy,
// yz, zz), q = sum (v-u) |v-u|^2/2 F w; zero for solid cells
__global__ void __launch_bounds__(256) k_momout3d(Geo3D G, const double* __restrict__ st,
                                                 double* __restrict__ out, double vmin, double dv,
                                                 double w) {
  __shared__ double lds[4];
  const int c = blockIdx.x;
  const int N = G.N, nvel = G.nvel;
  double* o = out + (size_t)c * 14;
  if (G.type[c] == TYPE_SOLID) {
    if (threadIdx.x < 14) o[threadIdx.x] = 0.0;
    return;
  }
  const double* f = st + (size_t)c * nvel;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
  for (int p = threadIdx.x; p < nvel; p += blockDim.x) {
    const double vx = vnode3(vmin, dv, p % N), vy = vnode3(vmin, dv, (p / N) % N),
                 vz = vnode3(vmin, dv, p / (N * N));
    s0 += f[p]; s1 += vx * f[p]; s2 += vy * f[p]; s3 += vz * f[p];
    s4 += (vx * vx + vy * vy + vz * vz) * f[p];
  }
  s0 = block_sum(s0, lds); s1 = block_sum(s1, lds); s2 = block_sum(s2, lds);
  s3 = block_sum(s3, lds); s4 = block_sum(s4, lds);
  const double rho = s0 * w, ux = s1 * w / rho, uy = s2 * w / rho, uz = s3 * w / rho;
  const double T = (2.0 * (0.5 * s4 * w) / rho - (ux * ux + uy * uy + uz * uz)) / 3.0;
  double a[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int p = threadIdx.x; p < nvel; p += blockDim.x) {
    const double cx = vnode3(vmin, dv, p % N) - ux, cy = vnode3(vmin, dv, (p / N) % N) - uy,
                 cz = vnode3(vmin, dv, p / (N * N)) - uz;
    const double fp = f[p];
    a[0] += cx * cx * fp; a[1] += cx * cy * fp; a[2] += cx * cz * fp;
    a[3] += cy * cy * fp; a[4] += cy * cz * fp; a[5] += cz * cz * fp;
    const double e = 0.5 * (cx * cx + cy * cy + cz * cz) * fp;
    a[6] += cx * e; a[7] += cy * e; a[8] += cz * e;
  }
  for (int u = 0; u < 9; ++u) a[u] = block_sum(a[u], lds) * w;
  if (threadIdx.x == 0) {
    o[0] = rho; o[1] = ux; o[2] = uy; o[3] = uz; o[4] = T;
    for (int u = 0; u < 9; ++u) o[5 + u] = a[u];
  }
}

// mass of the current state: one wave per cell, masters only; block partials
__global__ void __launch_bounds__(256) k_mass3d(Geo3D G, const double* __restrict__ st,
                                               double* __restrict__ mpart, double w) {
  __shared__ double lds[4];
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  if (c < G.ncell && G.master[c] == c)
    for (int p = lane; p < G.nvel; p += kWave) s += st[(size_t)c * G.nvel + p];
  s = wave_sum3(s);
  const double v = (c < G.ncell && G.master[c] == c) ? G.vcv[c] * s * w : 0.0;
  __syncthreads();
  if (lane == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) mpart[blockIdx.x] = ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

int node_count(int nvel) {
  int N = (int)llround(cbrt((double)nvel));
  return N * N * N == nvel ? N : 0;
}

typedef void (*step3_fn)(const Step3Args);
typedef void (*part3_fn)(Geo3D, const double*, double*, double, double);

template <int N>
void pick3(step3_fn* s, part3_fn* p, int* nch) {
  if (s) *s = k_step3d<N>;
  if (p) *p = k_part3d<N>;
  if (nch) *nch = Chunk3<N>::NCH;
}

bool select3(int N, step3_fn* s, part3_fn* p, int* nch) {
  switch (N) {
    case 4: pick3<4>(s, p, nch); return true;
    case 6: pick3<6>(s, p, nch); return true;
    case 8: pick3<8>(s, p, nch); return true;
    case 12: pick3<12>(s, p, nch); return true;
    case 16: pick3<16>(s, p, nch); return true;
    default: return false;
  }
}

double tau_coef(const cc_ctx* ctx) {
  return ctx->cfg.kn > 0.0 ? sqrt(M_PI) / 2.0 * ctx->cfg.kn * ctx->cfg.lref / sqrt(2.0) : 0.0;
}

double weight3(const cc_ctx* ctx) { return ctx->dv * ctx->dv * ctx->dv; }

int mom_blocks(const cc_ctx* ctx) { return (ctx->ncell + 255) / 256; }

hipError_t run_mom3d(cc_ctx* ctx) {
  Mom3Params P;
  P.w = weight3(ctx);
  P.dt = ctx->dt;
  P.tau_coef = tau_coef(ctx);
  P.vol = ctx->dx * ctx->dy * ctx->dz;
  P.nch = chunks3d(ctx->N);
  prof_begin(ctx, 4);
  k_mom3d<<<mom_blocks(ctx), 256, 0, ctx->stream>>>(ctx->g3, ctx->s.part, ctx->s.mom, ctx->s.mpart, P);
  prof_end(ctx, 4);
  return hipGetLastError();
}

Cut3Params cut_params(const cc_ctx* ctx, int write) {
  Cut3Params P;
  P.vmin = ctx->cfg.vmin;
  P.dv = ctx->dv;
  P.w = weight3(ctx);
  P.dt = ctx->dt;
  P.tau_coef = tau_coef(ctx);
  P.t_wall = ctx->body.t_wall;
  P.write_state = write;
  return P;
}

// force (and mass) slots of the current merged state into row[0..3]
hipError_t cut_and_reduce(cc_ctx* ctx, const double* in, double* out, int write, double* row) {
  const int nb = mom_blocks(ctx);
  double* mcut = ctx->s.mpart + nb;
  if (ctx->n_irr > 0) {
    prof_begin(ctx, 1);
    k_cut3d<<<ctx->n_irr, 256, 0, ctx->stream>>>(ctx->g3, in, out, ctx->s.fslot, mcut,
                                                 cut_params(ctx, write));
    prof_end(ctx, 1);
  }
  if (row) {
    prof_begin(ctx, 2);
    k_reduce3d<<<1, 256, 0, ctx->stream>>>(ctx->s.fslot, ctx->n_irr, ctx->s.mpart, nb, mcut, row);
    prof_end(ctx, 2);
  }
  return hipGetLastError();
}

}  // namespace

int chunks3d(int N) {
  int nch = 0;
  return select3(N, nullptr, nullptr, &nch) ? nch : 0;
}

bool regular_supported_3d(int nvel) {
  const int N = node_count(nvel);
  return N > 0 && select3(N, nullptr, nullptr, nullptr);
}

hipError_t launch_init_maxwellian_3d(cc_ctx* ctx) {
  const size_t tot = (size_t)ctx->ncell * ctx->nvel;
  k_init3d<<<(unsigned)((tot + 255) / 256), 256, 0, ctx->stream>>>(ctx->g3,
                                                                   (double*)ctx->state[ctx->cur]);
  return hipGetLastError();
}

hipError_t launch_load_state_3d(cc_ctx* ctx, const double* f) {
  const size_t tot = (size_t)ctx->ncell * ctx->nvel;
  k_load3d<<<(unsigned)((tot + 255) / 256), 256, 0, ctx->stream>>>(
      ctx->g3, (double*)ctx->state[ctx->cur], f);
  return hipGetLastError();
}

hipError_t launch_store_state_3d(const cc_ctx* ctx, double* f) {
  return hipMemcpyAsync(f, ctx->state[ctx->cur], (size_t)ctx->ncell * ctx->nvel * sizeof(double),
                        hipMemcpyDeviceToDevice, ctx->stream);
}

hipError_t launch_merge_3d(cc_ctx* ctx) {
  if (ctx->n_irr == 0) return hipSuccess;
  prof_begin(ctx, 3);
  k_merge3d<<<ctx->n_irr, 256, 0, ctx->stream>>>(ctx->g3, (double*)ctx->state[ctx->cur]);
  prof_end(ctx, 3);
  return hipGetLastError();
}

hipError_t launch_moments_all_3d(cc_ctx* ctx) {
  part3_fn fn = nullptr;
  if (!select3(ctx->N, nullptr, &fn, nullptr)) return hipErrorNotSupported;
  fn<<<(ctx->ncell + 3) / 4, 256, 0, ctx->stream>>>(ctx->g3, (const double*)ctx->state[ctx->cur],
                                                     ctx->s.part, ctx->cfg.vmin, ctx->dv);
  return hipGetLastError();
}

// One step state[cur] -> state[1-cur]; row (nullable) = Fx, Fy, Fz, mass of
// the state entering the step.
hipError_t launch_step_3d(cc_ctx* ctx, double* row, double*) {
  step3_fn fn = nullptr;
  if (!select3(ctx->N, &fn, nullptr, nullptr)) return hipErrorNotSupported;
  hipError_t e = run_mom3d(ctx);
  if (e != hipSuccess) return e;
  const double* in = (const double*)ctx->state[ctx->cur];
  double* out = (double*)ctx->state[1 - ctx->cur];
  Step3Args A;
  A.in = in;
  A.out = out;
  A.kind = ctx->g3.kind;
  A.mom = ctx->s.mom;
  A.part = ctx->s.part;
  A.ghost = ctx->g3.ghost;
  A.nx = ctx->nx; A.ny = ctx->ny; A.nz = ctx->nz; A.nvel = ctx->nvel;
  A.ntj = (ctx->ny + kTY - 1) / kTY;
  A.ntiles = A.ntj * ((ctx->nz + kTZ - 1) / kTZ);
  A.nblk = A.ntiles * chunks3d(ctx->N);
  A.per = (A.nblk + 7) / 8;
  A.vmin = ctx->cfg.vmin;
  A.dv = ctx->dv;
  A.cxf = ctx->dt / ctx->dx; A.cyf = ctx->dt / ctx->dy; A.czf = ctx->dt / ctx->dz;
  prof_begin(ctx, 0);
  fn<<<A.per * 8, 1024, 0, ctx->stream>>>(A);
  prof_end(ctx, 0);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = cut_and_reduce(ctx, in, out, 1, row);
  if (e != hipSuccess) return e;
  ctx->cur = 1 - ctx->cur;
  ctx->nstep += 1;
  return hipSuccess;
}

hipError_t launch_mass_3d(cc_ctx* ctx, double* mass_row) {
  const int nb = (ctx->ncell + 3) / 4;
  k_mass3d<<<nb, 256, 0, ctx->stream>>>(ctx->g3, (const double*)ctx->state[ctx->cur], ctx->s.mpart,
                                         weight3(ctx));
  k_reduce3d<<<1, 256, 0, ctx->stream>>>(ctx->s.fslot, 0, ctx->s.mpart, nb, ctx->s.mpart, ctx->s.red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(mass_row, ctx->s.red + 3, sizeof(double), hipMemcpyDeviceToDevice,
                        ctx->stream);
}

hipError_t launch_moments_out_3d(cc_ctx* ctx, double* out) {
  k_momout3d<<<ctx->ncell, 256, 0, ctx->stream>>>(ctx->g3, (const double*)ctx->state[ctx->cur], out,
                                                   ctx->cfg.vmin, ctx->dv, weight3(ctx));
  return hipGetLastError();
}

// force and mass of the current (merged) state
hipError_t launch_force_only_3d(cc_ctx* ctx, double* out4) {
  hipError_t e = run_mom3d(ctx);
  if (e != hipSuccess) return e;
  return cut_and_reduce(ctx, (const double*)ctx->state[ctx->cur], nullptr, 0, out4);
}

}  // namespace ccdvm
