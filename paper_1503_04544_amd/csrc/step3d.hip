// Device step of the 3D cut-cell scheme (Section 5, eq. eq-schema3D, fixed
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
#include "equilibrium.h"

namespace ccdvm {
namespace {

constexpr int kWave = 64;
constexpr int kTY = 4, kTZ = 4, kTileWaves = kTY * kTZ;
// Own cells are loaded kPD3 + 2 x-steps before they are updated, halo cells
// kHaloPD x-steps before.  Vector-memory completions are waited for in issue
// order, so each x-step issues the halo loads (needed soonest) before the own
// prefetch.
constexpr int kPD3 = 2;
constexpr int kHaloPD = 0;
constexpr int kR16 = 4;   // velocities per lane of the N = 16 kernel

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

// Velocity sums of F kept per control volume and chunk: F, v F, |v|^2 F
// (kSums5) and, for the Shakhov model, v v^T F (xx, xy, xz, yy, yz, zz) and
// |v|^2 v F, from which the heat flux follows in one pass (kSumsSK).
constexpr int kSums5 = 5, kSumsSK = 14;
template <bool SK>
struct Sums3 {
  static constexpr int K = SK ? kSumsSK : kSums5;
  double s[K];
  __device__ inline Sums3() {
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = 0.0;
  }
  __device__ inline void add(double vx, double vy, double vz, double f) {
    const double v2 = vx * vx + vy * vy + vz * vz;
    s[0] += f; s[1] += vx * f; s[2] += vy * f; s[3] += vz * f;
    s[4] += v2 * f;
    if (SK) {
      s[5 + 0] += vx * vx * f; s[5 + 1] += vx * vy * f; s[5 + 2] += vx * vz * f;
      s[5 + 3] += vy * vy * f; s[5 + 4] += vy * vz * f; s[5 + 5] += vz * vz * f;
      s[11] += vx * v2 * f; s[12] += vy * v2 * f; s[13] += vz * v2 * f;
    }
  }
  template <class Red>
  __device__ inline void reduce(Red red) {
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = red(s[k]);
  }
};

// 3D Shakhov equilibrium (Section 2.1) from the Maxwellian value M at v,
// c = v - u: M [1 + (c.qt)(|c|^2/T - 5)], with the stored
// qt = (1 - Pr) q / (5 P T), P = rho T (R = 1).
__device__ inline double shakhov3(const double* __restrict__ qt, double invT, double cx, double cy,
                                  double cz, double M) {
  const double s = cx * qt[0] + cy * qt[1] + cz * qt[2];
  return M * (1.0 + s * ((cx * cx + cy * cy + cz * cz) * invT - 5.0));
}

// Chunking of the velocity set for N nodes per axis (N even, symmetric box).
template <int N>
struct Chunk3 {
  static constexpr int H = N / 2;                 // p2 (or p3) values of one sign
  static constexpr int E1 = H * N;                // velocities of one (p3, half of p2)
  // p3 per chunk (N = 16: as the dedicated kernel's chunks)
  static constexpr int G3 = N == 16 ? kR16 / 2 : ((H % 2 == 0) ? 2 : (H % 3 == 0 ? 3 : 1));
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
  double* part;         // per cell and chunk: the sums of Sums3 (5, Shakhov 14)
  const double* heat;   // Shakhov: (1 - Pr) q / (5 P T) per cell (3)
  const double* ghost;  // farfield values
  int nx, ny, nz, nvel;
  int ntj, ntiles, nblk, per;
  int ch0;              // first chunk of this launch
  int relax;            // 0: transport only (semi-implicit step)
  double vmin, dv, cxf, cyf, czf;   // dt/dx, dt/dy, dt/dz
};

template <int N, bool SK>
__global__ void __launch_bounds__(1024) k_step3d(const Step3Args A, const int* __restrict__ kind,
                                                const double* __restrict__ mom) {
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
  const int lch = logical / A.ntiles, tile = logical - lch * A.ntiles;
  const int ch = A.ch0 + lch;
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
  auto load_halo = [&](double (&hy)[R], double (&hz)[R], int i, int lv) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool a = active(lv, r);
      const int o = offset(lv, r);
      hy[r] = y_glob && a ? y_base[(size_t)i * y_step + o] : 0.0;
      hz[r] = z_glob && a ? z_base[(size_t)i * z_step + o] : 0.0;
    }
  };
  double hqy[kHaloPD + 1][R], hqz[kHaloPD + 1][R];
#pragma unroll
  for (int d = 0; d < kHaloPD; ++d) {
    if (d < nx) load_halo(hqy[d], hqz[d], d, lane);
    else
#pragma unroll
      for (int r = 0; r < R; ++r) { hqy[d][r] = 0.0; hqz[d][r] = 0.0; }
  }
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
    // prefetch: halos of cell i+kHaloPD, then own cell i+kPD3+2 (the
    // farfield past the end)
    if (i + kHaloPD < nx) load_halo(hqy[kHaloPD], hqz[kHaloPD], i + kHaloPD, lv);
    else
#pragma unroll
      for (int r = 0; r < R; ++r) { hqy[kHaloPD][r] = 0.0; hqz[kHaloPD][r] = 0.0; }
    double qn[R];
    const int ia = i + kPD3 + 2;
    if (ia <= nx) load_row(qn, own_row(ia), lv);
    else
#pragma unroll
      for (int r = 0; r < R; ++r) qn[r] = 0.0;
    const int s = i & 1;
#pragma unroll
    for (int r = 0; r < R; ++r) xch[s][wave][r][lv] = cur[r];
    __syncthreads();
    const int c = (int)(pencil + i);
    if (valid && kind[c] == KIND_REGULAR) {
      const double* mc = mom + 8 * (size_t)c;
      const double Am = mc[0], ux = mc[1], uy = mc[2], uz = mc[3], inv2T = mc[4];
      const double nu = A.relax ? mc[5] : 0.0;
      const double* qt = A.heat + 3 * (size_t)c;
      double tx = 0.0, tyy = 0.0, tzz = 0.0;
      if (lv < N) {
        const double v = vnode3(vmin, dv, lv);
        tx = exp(-(v - ux) * (v - ux) * inv2T);
        tyy = exp(-(v - uy) * (v - uy) * inv2T);
        tzz = exp(-(v - uz) * (v - uz) * inv2T);
      }
      Sums3<SK> sm;
      double* orow = A.out + (pencil + i) * (size_t)nvel;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = min(r * kWave + lv, C::CH - 1);
        const int rem = e % C::E1;
        const int p1 = rem % N, p2 = sy * C::H + rem / N, p3 = p3b + e / C::E1;
        const double vx = vnode3(vmin, dv, p1), vy = vnode3(vmin, dv, p2), vz = vnode3(vmin, dv, p3);
        double E = Am * __shfl(tx, p1, kWave) * __shfl(tyy, p2, kWave) * __shfl(tzz, p3, kWave);
        if (SK) E = shakhov3(qt, 2.0 * inv2T, vx - ux, vy - uy, vz - uz, E);
        const double yv = y_lds ? xch[s][wy][r][lv] : hqy[0][r];
        const double zv = z_lds ? xch[s][wz][r][lv] : hqz[0][r];
        const double f = cur[r];
        const double fxu = p1 >= C::H ? prv[r] : q[0][r];
        const double fn = f - A.cxf * fabs(vx) * (f - fxu) - A.cyf * fabs(vy) * (f - yv) -
                          A.czf * fabs(vz) * (f - zv) + nu * (E - f);
        if (active(lv, r)) {
          __builtin_nontemporal_store(fn, &orow[offset(lv, r)]);
          sm.add(vx, vy, vz, fn);
        }
      }
      sm.reduce([](double v) { return wave_sum3(v); });
      if (lv == 0) {
        double* pp = A.part + ((size_t)c * C::NCH + ch) * Sums3<SK>::K;
#pragma unroll
        for (int q2 = 0; q2 < Sums3<SK>::K; ++q2) pp[q2] = sm.s[q2];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      prv[r] = cur[r];
      cur[r] = q[0][r];
#pragma unroll
      for (int d = 0; d < kPD3; ++d) q[d][r] = q[d + 1][r];
      q[kPD3][r] = qn[r];
#pragma unroll
      for (int d = 0; d < kHaloPD; ++d) { hqy[d][r] = hqy[d + 1][r]; hqz[d][r] = hqz[d + 1][r]; }
    }
  }
}

// ---------------------------------------------------------------------
// N = 16 regular-cell kernel.  Same chunks as Chunk3<16> (R = 4 slots per
// lane, 16 chunks of 256 velocities), with the index structure made
// explicit: slot r of lane l holds p1 = l % 16, p2 = 8 sy + l / 16 +
// 4 (r & 1), p3 = p3b + r / 2, at offset (p3b + r/2) 256 + 128 sy +
// 64 (r & 1) + l in the cell.  Per x-step and wave: one exp per lane (lanes
// 0-15, 16-31, 32-47 build the x, y, z factors of the separable
// Maxwellian), the update written as c0 f + a_x f_x + a_y f_y + a_z f_z +
// (dt/tau) E, the five moment sums reduced by a reduce-scatter butterfly.
// Each wave publishes its cell in its LDS slot before the x-step barrier and
// then reads it back from there, as it reads the previous cell (x-upwind for
// v_x > 0) from its slot of the last x-step; so the own cells rotate through
// two register slots (next, in flight) and the x loop is unrolled by two.
// Halo cells of the next x-step are requested after the update.
// ---------------------------------------------------------------------
constexpr int kG16 = kR16 / 2;           // p3 values per chunk
constexpr int kNCH16 = 2 * 16 / kG16;    // chunks

__device__ inline double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sums of v[0..4] over the wave: on return lanes 8q .. 8q+7 hold the sum
// of quantity q (q < 5).  Each level halves the quantities a lane keeps and
// adds its partner's copy of them; the last three levels sum within 8 lanes.
__device__ inline double reduce5(const double (&v)[5], int lv) {
  const bool b3 = lv & 8;
  double w[4];
  w[0] = pl32_sum(v[0], v[4]);   // lower half: quantity 0, upper half: 4
#pragma unroll
  for (int k = 1; k < 4; ++k) w[k] = pl32_sum(v[k], 0.0);
  double x[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) x[k] = pl16_sum(w[k], w[k + 2]);
  const double keep = b3 ? x[1] : x[0], send = b3 ? x[0] : x[1];
  double y = keep + dpp_d<kMirror16>(send);
  y += dpp_d<kMirror8>(y);
  y += dpp_d<kSwap2>(y);
  y += dpp_d<kSwap1>(y);
  return y;
}

// Sums of v[0..15] over the wave: on return lanes 4q .. 4q+3 hold the sum
// of quantity q.  Each level halves the quantities a lane keeps and adds its
// partner's copy of them.
__device__ inline double reduce16(const double (&v)[16], int lv) {
  const bool b3 = lv & 8, b2 = lv & 4;
  double a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = pl32_sum(v[k], v[k + 8]);
  double b[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) b[k] = pl16_sum(a[k], a[k + 4]);
  double c[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double keep = b3 ? b[k + 2] : b[k], send = b3 ? b[k] : b[k + 2];
    c[k] = keep + dpp_d<kMirror16>(send);
  }
  const double keep = b2 ? c[1] : c[0], send = b2 ? c[0] : c[1];
  double d = keep + dpp_d<kMirror8>(send);
  d += dpp_d<kSwap2>(d);
  d += dpp_d<kSwap1>(d);
  return d;
}

// e^x for the per-axis Maxwellian factors, table-driven (P. T. P. Tang,
// ACM TOMS 15(2), 1989): x = (32 m + j) ln2/32 + r with |r| <= ln2/64, so
// e^x = 2^m 2^(j/32) e^r; e^r from its degree-6 Taylor polynomial (the
// remainder is below 4e-18) and 2^(j/32) from a 32-entry table in LDS.
// ln2/32 is split into a 30-bit head (n * head is exact) and a tail.
// About 14 VALU operations against ~30 for the library exp; measured error
// on the CPU against libm below 1.5 ulp.
constexpr double kExpInvL = 46.16624130844683;       // 32 / ln2
constexpr double kExpLHi = 0.021660849364707246;     // ln2/32, 30 bits
constexpr double kExpLLo = 2.7791044496520866e-11;   // ln2/32 - kExpLHi
__device__ inline double exp_tab(double x, const double* __restrict__ tab) {
  const double n = rint(x * kExpInvL);
  const double r = fma(-n, kExpLLo, fma(-n, kExpLHi, x));
  double p = fma(r, 1.0 / 720.0, 1.0 / 120.0);
  p = fma(r, p, 1.0 / 24.0);
  p = fma(r, p, 1.0 / 6.0);
  p = fma(r, p, 0.5);
  p = fma(r, p, 1.0);
  p = fma(r, p, 1.0);
  const int ni = (int)n;
  return ldexp(tab[ni & 31] * p, ni >> 5);
}

struct Ctx16 {
  size_t pencil;          // cell index of the pencil's first cell
  const double* own_base;
  const double* y_base;
  const double* z_base;
  size_t y_step, z_step;
  int cbase, wy, wz, wave, p3b, sy, ch;
  bool valid, y_lds, z_lds, y_glob, z_glob;
};

constexpr int rof16(int r) { return (r >> 1) * 256 + (r & 1) * 64; }

// a double known to be the same in every lane, as a scalar value
__device__ inline double uniform_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// load from a wave-uniform base plus a per-lane unsigned byte offset, so
// that the address stays a scalar base + 32-bit lane offset
__device__ inline double ld_u(const double* base, unsigned lane_bytes) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + lane_bytes);
}

// halo cells i of the neighbouring tiles (or the farfield), for the waves
// on the upwind edges of the tile, each direction only where it is read
// (the kernel is sensitive to the number of memory requests: loading both
// directions on every edge wave, so that the registers are always written,
// cost 2.6 %)
__device__ __forceinline__ void load_halos16(const Ctx16& X, int i, int nx, unsigned lb,
                                             double (&hy)[kR16], double (&hz)[kR16]) {
  if (i >= nx) return;
  if (X.y_glob) {
    const double* ry = X.y_base + (size_t)i * X.y_step + X.cbase;
#pragma unroll
    for (int r = 0; r < kR16; ++r) hy[r] = ld_u(ry + rof16(r), lb);
  }
  if (X.z_glob) {
    const double* rz = X.z_base + (size_t)i * X.z_step + X.cbase;
#pragma unroll
    for (int r = 0; r < kR16; ++r) hz[r] = ld_u(rz + rof16(r), lb);
  }
}

template <int U, bool SK>
__device__ __forceinline__ void step16(const Step3Args& A, const int* __restrict__ kind,
                                       const double* __restrict__ mom, const Ctx16& X, int i,
                                       double (&S)[2][kR16], double (&hy)[kR16], double (&hz)[kR16],
                                       double (*xch)[kTileWaves][kR16][kWave],
                                       const double* __restrict__ etab) {
  constexpr int R = kR16;
  const int nx = A.nx, nvel = A.nvel;
  int lv = threadIdx.x & 63;
  asm volatile("" : "+v"(lv));
  // publish cell i, then reuse its registers for cell i+2 (the farfield
  // past the end); the update reads cell i back from the wave's own slot
  double (&cur)[R] = S[U & 1];
  const double (&nxt)[R] = S[(U + 1) & 1];
  const int s = i & 1;
  const unsigned lb = (unsigned)lv * 8u;
#pragma unroll
  for (int r = 0; r < R; ++r) xch[s][X.wave][r][lv] = cur[r];
  if (i + 2 <= nx && X.valid) {
    const double* row = (i + 2 < nx ? X.own_base + (size_t)(i + 2) * nvel : A.ghost) + X.cbase;
#pragma unroll
    for (int r = 0; r < R; ++r) cur[r] = ld_u(row + rof16(r), lb);
  }
  __syncthreads();
  const int c = (int)(X.pencil + i);
  if (X.valid && kind[c] == KIND_REGULAR) {
    const double* mc = mom + 8 * (size_t)c;
    const double Am = uniform_d(mc[0]), inv2T = uniform_d(mc[4]);
    const double nu = A.relax ? uniform_d(mc[5]) : 0.0;
    const double ux = uniform_d(mc[1]), uy = uniform_d(mc[2]), uz = uniform_d(mc[3]);
    const double vmin = A.vmin, dv = A.dv;
    const int g = lv >> 4;
    const double ug = g == 0 ? ux : (g == 1 ? uy : uz);
    const double vt = vnode3(vmin, dv, lv & 15) - ug;
    const double t = exp_tab(-vt * vt * inv2T, etab);
    const int p2a = X.sy * 8 + (lv >> 4);
    const double ex = __shfl(t, lv & 15, kWave);
    const double eya = __shfl(t, 16 + p2a, kWave), eyb = __shfl(t, 20 + p2a, kWave);
    const double vx = vnode3(vmin, dv, lv & 15);
    const double vya = vnode3(vmin, dv, p2a), vyb = vnode3(vmin, dv, p2a + 4);
    const double ax = A.cxf * fabs(vx), aya = A.cyf * fabs(vya), ayb = A.cyf * fabs(vyb);
    const double base = 1.0 - nu - ax;
    const double Ax = Am * ex;
    const double Exa = Ax * eya, Exb = Ax * eyb;
    const bool xpos = (lv & 15) >= 8;
    double* orow = A.out + (size_t)c * nvel + X.cbase;
    // Shakhov: E *= 1 + (c.qt)(|c|^2/T - 5), split into the lane's x/y part
    // and the wave-uniform z part
    double qtz = 0.0, invT = 0.0, kxy[2] = {0.0, 0.0}, cxy2[2] = {0.0, 0.0};
    if (SK) {
      const double* qt = A.heat + 3 * (size_t)c;
      const double qtx = uniform_d(qt[0]), qty = uniform_d(qt[1]);
      qtz = uniform_d(qt[2]);
      invT = 2.0 * inv2T;
      const double cx = vx - ux;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double cy = (h ? vyb : vya) - uy;
        kxy[h] = cx * qtx + cy * qty;
        cxy2[h] = (cx * cx + cy * cy) * invT - 5.0;
      }
    }
    double fnv[kR16];
    double Aa = 0.0, Ab = 0.0, m3 = 0.0, m4z = 0.0;
#pragma unroll
    for (int q = 0; q < kG16; ++q) {
      const double ez = readlane_d(t, 32 + X.p3b + q);
      const double vz = vnode3(vmin, dv, X.p3b + q);
      const double az = A.czf * fabs(vz);
      double Bq = 0.0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = 2 * q + h;
        const double ay = h ? ayb : aya;
        double E = (h ? Exb : Exa) * ez;
        if (SK) {
          const double cz = vz - uz;
          E *= 1.0 + (kxy[h] + cz * qtz) * (cxy2[h] + cz * cz * invT);
        }
        const double fx = xpos ? xch[s ^ 1][X.wave][r][lv] : nxt[r];
        const double fy = X.y_lds ? xch[s][X.wy][r][lv] : hy[r];
        const double fz = X.z_lds ? xch[s][X.wz][r][lv] : hz[r];
        const double c0 = base - ay - az;
        const double fn = c0 * xch[s][X.wave][r][lv] + ax * fx + ay * fy + az * fz + nu * E;
        __builtin_nontemporal_store(
            fn, reinterpret_cast<double*>(reinterpret_cast<char*>(orow + rof16(r)) + lb));
        if (h) Ab += fn; else Aa += fn;
        Bq += fn;
        fnv[r] = fn;
      }
      m3 += vz * Bq;
      m4z += vz * vz * Bq;
    }
    const double s0 = Aa + Ab;
    if (!SK) {
      double m[5];
      m[0] = s0;
      m[1] = vx * s0;
      m[2] = vya * Aa + vyb * Ab;
      m[3] = m3;
      m[4] = vx * vx * s0 + (vya * vya * Aa + vyb * vyb * Ab) + m4z;
      const double tot = reduce5(m, lv);
      if ((lv & 7) == 0 && lv < 40) A.part[((size_t)c * kNCH16 + X.ch) * kSums5 + (lv >> 3)] = tot;
    } else {
      // the 14 sums of Sums3 from the lane's values: v_x is the lane's, v_y
      // takes two values (vya in even slots, vyb in odd), v_z one per pair
      double yz = 0.0, y3z = 0.0, z3y = 0.0, z3 = 0.0;
#pragma unroll
      for (int q = 0; q < kG16; ++q) {
        const double vz = vnode3(vmin, dv, X.p3b + q);
        const double fa = fnv[2 * q], fb = fnv[2 * q + 1];
        const double yq = vya * fa + vyb * fb;          // sum v_y F over the pair
        yz += vz * yq;
        y3z += vz * vz * yq;
        z3y += vz * (vya * vya * fa + vyb * vyb * fb);
        z3 += vz * vz * vz * (fa + fb);
      }
      const double sy = vya * Aa + vyb * Ab, yy = vya * vya * Aa + vyb * vyb * Ab;
      const double vx2 = vx * vx;
      double m[16];
      m[0] = s0;
      m[1] = vx * s0;
      m[2] = sy;
      m[3] = m3;
      m[4] = vx2 * s0 + yy + m4z;
      m[5] = vx2 * s0;
      m[6] = vx * sy;
      m[7] = vx * m3;
      m[8] = yy;
      m[9] = yz;
      m[10] = m4z;
      m[11] = vx * m[4];
      m[12] = vx2 * sy + (vya * vya * vya * Aa + vyb * vyb * vyb * Ab) + y3z;
      m[13] = vx2 * m3 + z3y + z3;
      m[14] = 0.0;
      m[15] = 0.0;
      const double tot = reduce16(m, lv);
      if ((lv & 3) == 0 && lv < 4 * kSumsSK)
        A.part[((size_t)c * kNCH16 + X.ch) * kSumsSK + (lv >> 2)] = tot;
    }
  }
  // halos of cell i+1, once hy and hz are no longer read
  load_halos16(X, i + 1, nx, lb, hy, hz);
}

template <bool SK>
__global__ void __launch_bounds__(1024) k_step3d16(const Step3Args A, const int* __restrict__ kind,
                                                  const double* __restrict__ mom) {
  constexpr int R = kR16;
  __shared__ double xch[2][kTileWaves][R][kWave];
  __shared__ double etab[32];   // 2^(j/32); ordered before its first use by the first x-step's barrier
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x;
  const int logical = (b & 7) * A.per + (b >> 3);
  if (logical >= A.nblk) return;
  if (threadIdx.x < 32) etab[threadIdx.x] = exp2(threadIdx.x / 32.0);
  Ctx16 X;
  const int lch = logical / A.ntiles;
  const int tile = logical - lch * A.ntiles;
  X.ch = A.ch0 + lch;
  const int ty = wave & 3, tz = wave >> 2;
  const int tj = tile % A.ntj, tk = tile / A.ntj;
  const int j = tj * kTY + ty, k = tk * kTZ + tz;
  X.valid = j < A.ny && k < A.nz;
  X.sy = X.ch & 1;
  X.p3b = (X.ch >> 1) * kG16;
  X.wave = wave;
  X.cbase = X.p3b * 256 + X.sy * 128;
  const int dyu = X.sy ? -1 : 1, dzu = X.p3b >= 8 ? -1 : 1;
  const int jy = j + dyu, kz = k + dzu, tyu = ty + dyu, tzu = tz + dzu;
  const bool y_dom = jy >= 0 && jy < A.ny, z_dom = kz >= 0 && kz < A.nz;
  X.y_lds = y_dom && tyu >= 0 && tyu < kTY;
  X.z_lds = z_dom && tzu >= 0 && tzu < kTZ;
  X.wy = X.y_lds ? tz * kTY + tyu : 0;
  X.wz = X.z_lds ? tzu * kTY + ty : 0;
  const int nx = A.nx, nvel = A.nvel;
  const size_t pencil = (size_t)((X.valid ? k : 0) * A.ny + (X.valid ? j : 0)) * nx;
  X.pencil = pencil;
  X.own_base = A.in + pencil * nvel;
  X.y_glob = X.valid && !X.y_lds;
  X.z_glob = X.valid && !X.z_lds;
  const bool yg = X.y_glob && y_dom, zg = X.z_glob && z_dom;
  X.y_base = yg ? A.in + (size_t)(k * A.ny + jy) * nx * nvel : A.ghost;
  X.z_base = zg ? A.in + (size_t)(kz * A.ny + j) * nx * nvel : A.ghost;
  X.y_step = yg ? nvel : 0;
  X.z_step = zg ? nvel : 0;
  double S[2][R], hy[R], hz[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int o = X.cbase + rof16(r) + lane;
    // cells 0 and 1 (the farfield past the end); x-upwind of cell 0 and the
    // halos of cell 0
    S[0][r] = X.valid ? X.own_base[o] : 0.0;
    S[1][r] = X.valid ? (1 < nx ? X.own_base[(size_t)nvel + o] : A.ghost[o]) : 0.0;
    xch[1][wave][r][lane] = X.valid ? A.ghost[o] : 0.0;
    hy[r] = 0.0;
    hz[r] = 0.0;
  }
  load_halos16(X, 0, nx, (unsigned)lane * 8u, hy, hz);
  for (int i = 0; i < nx; i += 2) {
    step16<0, SK>(A, kind, mom, X, i, S, hy, hz, xch, etab);
    if (i + 1 < nx) step16<1, SK>(A, kind, mom, X, i + 1, S, hy, hz, xch, etab);
  }
}

// partial moments of the current (merged) state, per control-volume master
// and chunk (one wave per cell)
template <int N, bool SK>
__global__ void __launch_bounds__(256) k_part3d(Geo3D G, const double* __restrict__ in,
                                               double* __restrict__ part, double vmin, double dv) {
  using C = Chunk3<N>;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= G.ncell || (G.kind[c] != KIND_REGULAR && G.kind[c] != KIND_IRREGULAR)) return;
  const double* row = in + (size_t)c * G.nvel;
  for (int ch = 0; ch < C::NCH; ++ch) {
    const int sy = ch & 1, p3b = (ch >> 1) * C::G3;
    Sums3<SK> sm;
    for (int r = 0; r < C::R; ++r) {
      const int e = r * kWave + lane;
      if (e >= C::CH) continue;
      const int rem = e % C::E1;
      const double vx = vnode3(vmin, dv, rem % N), vy = vnode3(vmin, dv, sy * C::H + rem / N),
                   vz = vnode3(vmin, dv, p3b + e / C::E1);
      sm.add(vx, vy, vz, row[chunk_offset<N>(ch, e)]);
    }
    sm.reduce([](double v) { return wave_sum3(v); });
    if (lane == 0) {
      double* pp = part + ((size_t)c * C::NCH + ch) * Sums3<SK>::K;
      for (int q = 0; q < Sums3<SK>::K; ++q) pp[q] = sm.s[q];
    }
  }
}

struct Mom3Params {
  double w, dt, tau_coef, vol;
  double vmin, dv;
  int nch, N;
  int conservative;     // conservative equilibrium (Section 3.1)
  // 0: explicit step (equilibrium and dt/tau from the same triplet);
  // 1: semi-implicit step at t^n (dt/tau from the direct density only);
  // 2: semi-implicit step, equilibrium of the transported value (dt/tau of
  //    t^n kept)
  int mode;
  double sk_coef;       // Shakhov: (1 - Pr)/5
};

// moments of every control volume from its chunk sums (eq. MacroscopicTD):
// rho, u, T = (2E/rho - |u|^2)/3 (or the conservative triplet), the
// relaxation record, block partials of the mass sum_m V_m rho_m and, for
// the Shakhov model, the heat flux about the direct mean velocity,
//   q = 1/2 [S3 - 2 S2 u - u tr S2 + 2 rho |u|^2 u],
// S2 = sum v v^T F w, S3 = sum |v|^2 v F w, stored as
// (1 - Pr) q / (5 rho T^2) with the triplet of the record
// Four lanes per control volume: lane j of a quad sums the chunks j, j + 4,
// ... (every chunk count is a multiple of 4), the quad adds its four sums
// through lane swaps (each lane ends with the same bits) and the record's
// slots are stored by the quad's lanes in turn, so a wave reads the sums of
// 16 consecutive control volumes and writes their records as whole rows.
// With the conservative triplet one thread per control volume: the Newton
// solve would otherwise run in all four lanes of the quad.
template <bool CONS, bool SK>
__global__ void __launch_bounds__(256) k_mom3d(Geo3D G, const double* __restrict__ part,
                                              double* __restrict__ mom, double* __restrict__ heat,
                                              double* __restrict__ mpart, Mom3Params P) {
  constexpr int K = Sums3<SK>::K;
  constexpr int CPT = CONS ? 1 : 4;   // threads per control volume
  __shared__ double lds[4];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = t / CPT, j = t % CPT;
  // the sums are requested together with the kind (from the last control
  // volume for the lanes past the end); those of other kinds are not used
  const int cc = c < G.ncell ? c : G.ncell - 1;
  const int kd = c < G.ncell ? G.kind[cc] : KIND_SOLID;
  double s[K];
#pragma unroll
  for (int q = 0; q < K; ++q) s[q] = 0.0;
  const double* pp = part + (size_t)cc * P.nch * K;
  for (int ch = j; ch < P.nch; ch += CPT)
#pragma unroll
    for (int q = 0; q < K; ++q) s[q] += pp[K * ch + q];
  const bool live = kd == KIND_REGULAR || kd == KIND_IRREGULAR;
  if (CPT == 4) {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      s[q] += dpp_d<kSwap1>(s[q]);
      s[q] += dpp_d<kSwap2>(s[q]);
    }
  }
  double ms = 0.0;
  if (live) {
    const double rho = s[0] * P.w;
    const double ux = s[1] * P.w / rho, uy = s[2] * P.w / rho, uz = s[3] * P.w / rho;
    const double en = 0.5 * s[4] * P.w;
    const double T = (2.0 * en / rho - (ux * ux + uy * uy + uz * uz)) / 3.0;
    double x[5] = {rho, ux, uy, uz, T};
    if (CONS && P.mode != 1) {
      const double target[5] = {rho, s[1] * P.w, s[2] * P.w, s[3] * P.w, en};
      if (!conservative_triplet_3d(x, target, P.vmin, P.dv, P.N)) {
        x[0] = rho; x[1] = ux; x[2] = uy; x[3] = uz; x[4] = T;
      }
    }
    // record slots: 0 density factor, 1-3 velocity, 4 1/(2T), 5 dt/tau, 6 rho
    const double r0 = x[0] / pow(2.0 * M_PI * x[4], 1.5);
    const double r5 = P.tau_coef > 0.0 ? P.dt * (P.mode == 1 ? rho : x[0]) / P.tau_coef : 0.0;
    double* mo = mom + 8 * (size_t)c;
#pragma unroll
    for (int sl = j; sl < 4; sl += CPT) mo[sl] = sl == 0 ? r0 : (sl == 1 ? x[1] : (sl == 2 ? x[2] : x[3]));
#pragma unroll
    for (int sl = j; sl < 3; sl += CPT)
      if (sl != 1 || P.mode != 2) mo[4 + sl] = sl == 0 ? 0.5 / x[4] : (sl == 1 ? r5 : rho);
    if (SK) {
      // heat flux component d from the row d of S2
      const double w = P.w, u2 = ux * ux + uy * uy + uz * uz;
      const double tr = s[5] * w + s[8] * w + s[10] * w;
      const double a = P.sk_coef / (x[0] * x[4] * x[4]);
#pragma unroll
      for (int d = j; d < 3; d += CPT) {
        const double r0x = d == 0 ? s[5] : (d == 1 ? s[6] : s[7]);
        const double r1x = d == 0 ? s[6] : (d == 1 ? s[8] : s[9]);
        const double r2x = d == 0 ? s[7] : (d == 1 ? s[9] : s[10]);
        const double s3 = d == 0 ? s[11] : (d == 1 ? s[12] : s[13]);
        const double ud = d == 0 ? ux : (d == 1 ? uy : uz);
        const double S2u = (r0x * w) * ux + (r1x * w) * uy + (r2x * w) * uz;
        const double qd = 0.5 * (s3 * w - 2.0 * S2u - ud * tr + 2.0 * rho * u2 * ud);
        heat[3 * (size_t)c + d] = a * qd;
      }
    }
    if (j == 0) ms = (kd == KIND_REGULAR ? P.vol : G.vcv[c]) * rho;
  }
  ms = block_sum(ms, lds);
  if (threadIdx.x == 0) mpart[blockIdx.x] = ms;
}

struct Cut3Params {
  double vmin, dv, w, dt, tau_coef, t_wall;
  int write_state;
  int conservative;     // conservative equilibrium (Section 3.1)
  int relax;            // 0: transport only (semi-implicit step)
};

// One control volume that is cut or owns merged cells: wall density of each
// wall face (zero net mass flux, Section 5), fluxes through the six
// Cartesian faces and the wall face of every member, explicit update with
// relaxation toward the Maxwellian of the control volume's record (built by
// k_mom3d), redistribution to the members, the moment sums of the new value
// (chunk slot 0) for the next record; wall stress -> force of the state at
// t^n.  write_state == 0: force only.
// Both Maxwellians are separable: their per-axis factors (N exponentials
// each) and the members' faces are set up in LDS once per block, so the
// velocity loops read tables instead of evaluating exponentials.
constexpr int kMaxN3 = 16;   // largest velocity nodes per axis of the 3D kernels
template <bool SK>
__global__ void __launch_bounds__(256) k_cut3d(Geo3D G, const double* __restrict__ in,
                                              double* __restrict__ out, double* __restrict__ fslot,
                                              const double* __restrict__ mom, const double* __restrict__ heat,
                                              double* __restrict__ part, int nch, Cut3Params P) {
  constexpr int K = Sums3<SK>::K;
  __shared__ double lds[4];
  __shared__ double wf[kMaxN3];                  // exp(-v^2 / (2 T_w))
  __shared__ double ef[3][kMaxN3];               // exp(-(v - u_d)^2 / (2 T))
  __shared__ double mS[kMaxMembers][6];          // members' Cartesian face areas
  __shared__ long long mnb[kMaxMembers][6];      // upwind neighbour's cell, -1: farfield
  __shared__ double mw[kMaxMembers][5];          // wall area, normal, density
  const int tid = threadIdx.x, nth = blockDim.x;
  const int q = blockIdx.x;
  const int m = G.irr[q];
  const int b = G.mptr[q], nm = min(G.mptr[q + 1] - b, kMaxMembers);
  const int N = G.N, nvel = G.nvel, nx = G.nx, ny = G.ny, nz = G.nz;
  const double* own = in + (size_t)m * nvel;
  const double* rec = mom + 8 * (size_t)m;
  const double Am = rec[0], ux = rec[1], uy = rec[2], uz = rec[3], inv2T = rec[4];
  const double nu = P.relax ? rec[5] : 0.0;
  const double* qt = SK ? heat + 3 * (size_t)m : nullptr;
  const double V = G.vcv[m];
  const double Tw = P.t_wall;
  const double cw = 1.0 / pow(2.0 * M_PI * Tw, 1.5);   // wall Maxwellian of unit density
  if (tid < N) {
    const double v = vnode3(P.vmin, P.dv, tid);
    wf[tid] = exp(-(v * v) / (2.0 * Tw));
    ef[0][tid] = exp(-(v - ux) * (v - ux) * inv2T);
    ef[1][tid] = exp(-(v - uy) * (v - uy) * inv2T);
    ef[2][tid] = exp(-(v - uz) * (v - uz) * inv2T);
  }
  if (tid < nm) {
    const int k = G.mem[b + tid];
    const int i = k % nx, j = (k / nx) % ny, kk = k / (nx * ny);
    const bool inside[6] = {i > 0, i + 1 < nx, j > 0, j + 1 < ny, kk > 0, kk + 1 < nz};
    const long long stride[3] = {1, nx, (long long)nx * ny};
    const double S[6] = {G.sxm[k], G.sxp[k], G.sym[k], G.syp[k], G.szm[k], G.szp[k]};
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      mS[tid][f] = S[f];
      mnb[tid][f] = inside[f] ? k + ((f & 1) ? stride[f >> 1] : -stride[f >> 1]) : -1;
    }
    mw[tid][0] = G.aw[k];
    mw[tid][1] = G.nwx[k];
    mw[tid][2] = G.nwy[k];
    mw[tid][3] = G.nwz[k];
    mw[tid][4] = 0.0;
  }
  __syncthreads();
  for (int t = 0; t < nm; ++t) {
    if (!(mw[t][0] > 0.0)) continue;
    const double n0 = mw[t][1], n1 = mw[t][2], n2 = mw[t][3];
    double num = 0.0, den = 0.0;
    // four velocities per thread at a time, their values requested together
    // (past the last velocity the thread's first one is read and not used)
    for (int p0 = tid; p0 < nvel; p0 += 4 * nth) {
      double o[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p = p0 + u * nth;
        o[u] = own[p < nvel ? p : p0];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p = p0 + u * nth;
        if (p >= nvel) continue;
        const int p1 = p % N, p2 = (p / N) % N, p3 = p / (N * N);
        const double vx = vnode3(P.vmin, P.dv, p1), vy = vnode3(P.vmin, P.dv, p2), vz = vnode3(P.vmin, P.dv, p3);
        const double cn = vx * n0 + vy * n1 + vz * n2;
        if (cn > 0.0) num += cn * o[u];
        else if (cn < 0.0) den += cn * (cw * (wf[p1] * wf[p2] * wf[p3]));
      }
    }
    num = block_sum(num, lds);
    den = block_sum(den, lds);
    if (tid == 0) mw[t][4] = den != 0.0 ? -num / den : 0.0;
  }
  __syncthreads();
  double Fx = 0.0, Fy = 0.0, Fz = 0.0;
  Sums3<SK> sm;
  for (int p = tid; p < nvel; p += nth) {
    const int p1 = p % N, p2 = (p / N) % N, p3 = p / (N * N);
    const double v[3] = {vnode3(P.vmin, P.dv, p1), vnode3(P.vmin, P.dv, p2), vnode3(P.vmin, P.dv, p3)};
    const double fo = own[p];
    const double Mw = cw * (wf[p1] * wf[p2] * wf[p3]);
    double Rs = 0.0;
    for (int t = 0; t < nm; ++t) {
      // the six faces' upwind values are requested together (a closed face
      // reads the cell's own value and adds a zero term)
      double fn[6];
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const long long nb = mnb[t][f];
        const double* src = !(mS[t][f] > 0.0) ? own : (nb >= 0 ? in + (size_t)nb * nvel : G.ghost);
        fn[f] = src[p];
      }
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const double S = mS[t][f] > 0.0 ? mS[t][f] : 0.0;
        const int d = f >> 1;
        const double cvel = (f & 1) ? v[d] : -v[d];   // outward normal velocity
        Rs += S * (fmax(cvel, 0.0) * fo + fmin(cvel, 0.0) * fn[f]);
      }
      const double aw = mw[t][0];
      if (aw > 0.0) {
        const double cn = v[0] * mw[t][1] + v[1] * mw[t][2] + v[2] * mw[t][3];
        const double fw = mw[t][4] * Mw;
        Rs += aw * (fmin(cn, 0.0) * fw + fmax(cn, 0.0) * fo);
        const double fv = cn < 0.0 ? fw : (cn > 0.0 ? fo : 0.0);
        const double s = aw * cn * fv;
        Fx += v[0] * s;
        Fy += v[1] * s;
        Fz += v[2] * s;
      }
    }
    if (P.write_state) {
      const double cx = v[0] - ux, cy = v[1] - uy, cz = v[2] - uz;
      double E = nu != 0.0 ? Am * (ef[0][p1] * ef[1][p2] * ef[2][p3]) : 0.0;
      if (SK && nu != 0.0) E = shakhov3(qt, 2.0 * inv2T, cx, cy, cz, E);
      const double fn = fo - P.dt / V * Rs + nu * (E - fo);
      for (int t = 0; t < nm; ++t) out[(size_t)G.mem[b + t] * nvel + p] = fn;
      sm.add(v[0], v[1], v[2], fn);
    }
  }
  if (P.write_state) {
    sm.reduce([&](double x) { return block_sum(x, lds); });
    double* pp = part + (size_t)m * nch * K;
    for (int k = tid; k < nch * K; k += nth) pp[k] = 0.0;
    __syncthreads();
    if (tid == 0)
      for (int k = 0; k < K; ++k) pp[k] = sm.s[k];
  }
  Fx = block_sum(Fx, lds) * P.w;
  Fy = block_sum(Fy, lds) * P.w;
  Fz = block_sum(Fz, lds) * P.w;
  if (tid == 0) {
    fslot[3 * q + 0] = Fx;
    fslot[3 * q + 1] = Fy;
    fslot[3 * q + 2] = Fz;
  }
}

// diag row: force summed over the control volumes in list order, mass over
// the block partials of the moment pass
__global__ void __launch_bounds__(256) k_reduce3d(const double* __restrict__ fslot, int ncv,
                                                 const double* __restrict__ mpart, int nmp,
                                                 double* __restrict__ row) {
  __shared__ double lds[4];
  double fx = 0.0, fy = 0.0, fz = 0.0, ms = 0.0;
  for (int t = threadIdx.x; t < ncv; t += blockDim.x) {
    fx += fslot[3 * t]; fy += fslot[3 * t + 1]; fz += fslot[3 * t + 2];
  }
  {
    // four partials in flight per thread
    const int bd = blockDim.x;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    int t = threadIdx.x;
    for (; t + 3 * bd < nmp; t += 4 * bd) {
      m0 += mpart[t]; m1 += mpart[t + bd]; m2 += mpart[t + 2 * bd]; m3 += mpart[t + 3 * bd];
    }
    for (; t < nmp; t += bd) m0 += mpart[t];
    ms = (m0 + m1) + (m2 + m3);
  }
  fx = block_sum(fx, lds); fy = block_sum(fy, lds); fz = block_sum(fz, lds);
  ms = block_sum(ms, lds);
  if (threadIdx.x == 0) {
    row[0] = fx; row[1] = fy; row[2] = fz;
    row[3] = ms;
  }
}

// merge over the control volumes with more than one member (Section 5
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

// Semi-implicit step, last part: every non-solid cell's transported value
// F* relaxes implicitly toward the equilibrium of its control volume's
// transported moments, F = (F* + nu E)/(1 + nu) (nu = dt/tau^n from the
// record), in place; masters also store the moment sums of the new value
// (chunk slot 0, the other slots zero).  One wave per cell; the separable
// Maxwellian is tabulated per axis in the first N lanes when the velocity
// count is a multiple of the wave.
template <int N, bool SK>
__global__ void __launch_bounds__(256) k_relax3d(Geo3D G, double* __restrict__ st,
                                                const double* __restrict__ mom,
                                                const double* __restrict__ heat,
                                                double* __restrict__ part, int nch, double vmin,
                                                double dv) {
  constexpr int K = Sums3<SK>::K;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= G.ncell) return;
  const int m = G.master[c];
  if (m < 0) return;
  constexpr int nvel = N * N * N;
  const double* rec = mom + 8 * (size_t)m;
  const double Am = rec[0], ux = rec[1], uy = rec[2], uz = rec[3], inv2T = rec[4], nu = rec[5];
  const double* qt = SK ? heat + 3 * (size_t)m : nullptr;
  const double sc = 1.0 / (1.0 + nu);
  double tx = 0.0, ty = 0.0, tz = 0.0;
  if (lane < N) {
    const double v = vnode3(vmin, dv, lane);
    tx = exp(-(v - ux) * (v - ux) * inv2T);
    ty = exp(-(v - uy) * (v - uy) * inv2T);
    tz = exp(-(v - uz) * (v - uz) * inv2T);
  }
  constexpr bool tables = nvel % kWave == 0;
  double* row = st + (size_t)c * nvel;
  Sums3<SK> sm;
  // eight independent loads per lane in flight, then their updates
  constexpr int B = 8;
  for (int p0 = 0; p0 < nvel; p0 += B * kWave) {
    double fv[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int p = p0 + u * kWave + lane;
      fv[u] = p < nvel ? row[p] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int p = p0 + u * kWave + lane;
      if (p >= nvel) continue;
      const int p1 = p % N, p2 = (p / N) % N, p3 = p / (N * N);
      const double vx = vnode3(vmin, dv, p1), vy = vnode3(vmin, dv, p2), vz = vnode3(vmin, dv, p3);
      double E;
      if (tables) {
        E = Am * __shfl(tx, p1, kWave) * __shfl(ty, p2, kWave) * __shfl(tz, p3, kWave);
      } else {
        const double cx = vx - ux, cy = vy - uy, cz = vz - uz;
        E = Am * exp(-(cx * cx + cy * cy + cz * cz) * inv2T);
      }
      if (SK) E = shakhov3(qt, 2.0 * inv2T, vx - ux, vy - uy, vz - uz, E);
      const double fn = (fv[u] + nu * E) * sc;
      __builtin_nontemporal_store(fn, &row[p]);
      sm.add(vx, vy, vz, fn);
    }
  }
  if (c != m) return;
  sm.reduce([](double x) { return wave_sum3(x); });
  double* pp = part + (size_t)c * nch * K;
  for (int k = lane; k < nch * K; k += kWave) pp[k] = 0.0;
  if (lane == 0)
    for (int k = 0; k < K; ++k) pp[k] = sm.s[k];
}

int node_count(int nvel) {
  int N = (int)llround(cbrt((double)nvel));
  return N * N * N == nvel ? N : 0;
}

typedef void (*step3_fn)(const Step3Args, const int*, const double*);
typedef void (*part3_fn)(Geo3D, const double*, double*, double, double);

template <int N, bool SK>
void pick3(step3_fn* s, part3_fn* p, int* nch) {
  if constexpr (N == 16) {
    if (s) *s = k_step3d16<SK>;
  } else {
    if (s) *s = k_step3d<N, SK>;
  }
  if (p) *p = k_part3d<N, SK>;
  if (nch) *nch = Chunk3<N>::NCH;
}

template <bool SK>
bool select3_sk(int N, step3_fn* s, part3_fn* p, int* nch) {
  switch (N) {
    case 4: pick3<4, SK>(s, p, nch); return true;
    case 6: pick3<6, SK>(s, p, nch); return true;
    case 8: pick3<8, SK>(s, p, nch); return true;
    case 12: pick3<12, SK>(s, p, nch); return true;
    case 16: pick3<16, SK>(s, p, nch); return true;
    default: return false;
  }
}

bool select3(int N, step3_fn* s, part3_fn* p, int* nch, bool sk = false) {
  return sk ? select3_sk<true>(N, s, p, nch) : select3_sk<false>(N, s, p, nch);
}


double tau_coef(const cc_ctx* ctx) {
  return ctx->cfg.kn > 0.0 ? sqrt(M_PI) / 2.0 * ctx->cfg.kn * ctx->cfg.lref / sqrt(2.0) : 0.0;
}

double weight3(const cc_ctx* ctx) { return ctx->dv * ctx->dv * ctx->dv; }

// blocks of the moment pass: 64 control volumes per block (four threads
// each), 256 with the conservative triplet (one thread each)
int mom_blocks(const cc_ctx* ctx) {
  return ctx->cfg.maxwellian == CC_MAXW_CONSERVATIVE ? (ctx->ncell + 255) / 256 : (ctx->ncell + 63) / 64;
}

hipError_t run_mom3d(cc_ctx* ctx, int mode = 0) {
  Mom3Params P;
  P.w = weight3(ctx);
  P.dt = ctx->dt;
  P.tau_coef = tau_coef(ctx);
  P.vol = ctx->dx * ctx->dy * ctx->dz;
  P.vmin = ctx->cfg.vmin;
  P.dv = ctx->dv;
  P.nch = chunks3d(ctx->N);
  P.N = ctx->N;
  P.conservative = ctx->cfg.maxwellian == CC_MAXW_CONSERVATIVE;
  P.mode = mode;
  P.sk_coef = (1.0 - ctx->cfg.prandtl) / 5.0;
  const bool sk = ctx->cfg.model == CC_MODEL_SHAKHOV;
  auto fn = P.conservative ? (sk ? k_mom3d<true, true> : k_mom3d<true, false>)
                           : (sk ? k_mom3d<false, true> : k_mom3d<false, false>);
  prof_begin(ctx, 4);
  fn<<<mom_blocks(ctx), 256, 0, ctx->stream>>>(ctx->g3, ctx->s.part, ctx->s.mom, ctx->s.heat, ctx->s.mpart, P);
  prof_end(ctx, 4);
  return hipGetLastError();
}

Cut3Params cut_params(const cc_ctx* ctx, int write, int relax = 1) {
  Cut3Params P;
  P.vmin = ctx->cfg.vmin;
  P.dv = ctx->dv;
  P.w = weight3(ctx);
  P.dt = ctx->dt;
  P.tau_coef = tau_coef(ctx);
  P.t_wall = ctx->body.t_wall;
  P.write_state = write;
  P.conservative = ctx->cfg.maxwellian == CC_MAXW_CONSERVATIVE;
  P.relax = relax;
  return P;
}

// force (and mass) slots of the current merged state into row[0..3]
hipError_t cut_and_reduce(cc_ctx* ctx, const double* in, double* out, int write, double* row,
                          int relax = 1) {
  const int nb = mom_blocks(ctx);
  if (ctx->n_irr > 0) {
    prof_begin(ctx, 1);
    auto fn = ctx->cfg.model == CC_MODEL_SHAKHOV ? k_cut3d<true> : k_cut3d<false>;
    fn<<<ctx->n_irr, 256, 0, ctx->stream>>>(ctx->g3, in, out, ctx->s.fslot, ctx->s.mom, ctx->s.heat,
                                            ctx->s.part, chunks3d(ctx->N), cut_params(ctx, write, relax));
    prof_end(ctx, 1);
  }
  if (row) {
    prof_begin(ctx, 2);
    k_reduce3d<<<1, 256, 0, ctx->stream>>>(ctx->s.fslot, ctx->n_irr, ctx->s.mpart, nb, row);
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
  if (!select3(ctx->N, nullptr, &fn, nullptr, ctx->cfg.model == CC_MODEL_SHAKHOV)) return hipErrorNotSupported;
  fn<<<(ctx->ncell + 3) / 4, 256, 0, ctx->stream>>>(ctx->g3, (const double*)ctx->state[ctx->cur],
                                                     ctx->s.part, ctx->cfg.vmin, ctx->dv);
  return hipGetLastError();
}

// One step state[cur] -> state[1-cur]; row (nullable) = Fx, Fy, Fz, mass of
// the state entering the step.
hipError_t launch_step_3d(cc_ctx* ctx, double* row, double*) {
  step3_fn fn = nullptr;
  if (!select3(ctx->N, &fn, nullptr, nullptr, ctx->cfg.model == CC_MODEL_SHAKHOV)) return hipErrorNotSupported;
  const bool imex = ctx->cfg.scheme == CC_SCHEME_IMEX;
  hipError_t e = run_mom3d(ctx, imex ? 1 : 0);
  if (e != hipSuccess) return e;
  const double* in = (const double*)ctx->state[ctx->cur];
  double* out = (double*)ctx->state[1 - ctx->cur];
  Step3Args A;
  A.in = in;
  A.out = out;
  A.kind = ctx->g3.kind;
  A.mom = ctx->s.mom;
  A.part = ctx->s.part;
  A.heat = ctx->s.heat;
  A.ghost = ctx->g3.ghost;
  A.nx = ctx->nx; A.ny = ctx->ny; A.nz = ctx->nz; A.nvel = ctx->nvel;
  A.ntj = (ctx->ny + kTY - 1) / kTY;
  A.ntiles = A.ntj * ((ctx->nz + kTZ - 1) / kTZ);
  A.nblk = A.ntiles * chunks3d(ctx->N);
  A.per = (A.nblk + 7) / 8;
  A.vmin = ctx->cfg.vmin;
  A.dv = ctx->dv;
  A.cxf = ctx->dt / ctx->dx; A.cyf = ctx->dt / ctx->dy; A.czf = ctx->dt / ctx->dz;
  A.relax = imex ? 0 : 1;
  // the cut control volumes and the force/mass reduction (disjoint cells,
  // their own slots) run on a side stream beside the streaming kernel;
  // serial while profiling
  const bool overlap = ctx->side && !ctx->prof.on;
  if (overlap) {
    e = hipEventRecord(ctx->fork, ctx->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(ctx->side, ctx->fork, 0);
    if (e != hipSuccess) return e;
    hipStream_t main = ctx->stream;
    ctx->stream = ctx->side;
    e = cut_and_reduce(ctx, in, out, 1, row, imex ? 0 : 1);
    ctx->stream = main;
    if (e != hipSuccess) return e;
    e = hipEventRecord(ctx->join, ctx->side);
    if (e != hipSuccess) return e;
  }
  prof_begin(ctx, 0);
  A.ch0 = 0;
  fn<<<A.per * 8, 1024, 0, ctx->stream>>>(A, A.kind, A.mom);
  prof_end(ctx, 0);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (overlap) {
    e = hipStreamWaitEvent(ctx->stream, ctx->join, 0);
  } else {
    e = cut_and_reduce(ctx, in, out, 1, row, imex ? 0 : 1);
  }
  if (e != hipSuccess) return e;
  if (imex) {
    // semi-implicit step (ImpSchemeDD): equilibrium of the transported
    // value, then the implicit relaxation in place
    e = run_mom3d(ctx, 2);
    if (e != hipSuccess) return e;
    prof_begin(ctx, 5);
    const bool sk = ctx->cfg.model == CC_MODEL_SHAKHOV;
    decltype(&k_relax3d<16, false>) rfn = nullptr;
    switch (ctx->N) {
      case 4: rfn = sk ? k_relax3d<4, true> : k_relax3d<4, false>; break;
      case 6: rfn = sk ? k_relax3d<6, true> : k_relax3d<6, false>; break;
      case 8: rfn = sk ? k_relax3d<8, true> : k_relax3d<8, false>; break;
      case 12: rfn = sk ? k_relax3d<12, true> : k_relax3d<12, false>; break;
      default: rfn = sk ? k_relax3d<16, true> : k_relax3d<16, false>; break;
    }
    rfn<<<(ctx->ncell + 3) / 4, 256, 0, ctx->stream>>>(ctx->g3, out, ctx->s.mom, ctx->s.heat, ctx->s.part,
                                                       chunks3d(ctx->N), ctx->cfg.vmin, ctx->dv);
    prof_end(ctx, 5);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  ctx->cur = 1 - ctx->cur;
  ctx->nstep += 1;
  return hipSuccess;
}

hipError_t launch_mass_3d(cc_ctx* ctx, double* mass_row) {
  const int nb = (ctx->ncell + 3) / 4;
  k_mass3d<<<nb, 256, 0, ctx->stream>>>(ctx->g3, (const double*)ctx->state[ctx->cur], ctx->s.mpart,
                                         weight3(ctx));
  k_reduce3d<<<1, 256, 0, ctx->stream>>>(ctx->s.fslot, 0, ctx->s.mpart, nb, ctx->s.red);
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
