// Internal declarations of the ccdvm library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string>
#include <vector>

#include "ccdvm.h"

namespace ccdvm {

// Per-cell kind used to dispatch the step.
enum CellKind : int {
  KIND_REGULAR = 0,    // gas cell, control volume of one cell: fused stencil kernel
  KIND_IRREGULAR = 1,  // master of a control volume that is cut or owns merged cells
  KIND_MEMBER = 2,     // non-master virtual cell: receives its master's value
  KIND_SOLID = 3
};

enum CellType : int { TYPE_GAS = 0, TYPE_CUT = 1, TYPE_SOLID = 2 };

// Maximum number of virtual cells merged into one control volume that the
// cut-cell kernel handles (the master search stops after 4 hops, and in the
// workloads a control volume holds at most 3 cells).
constexpr int kMaxMembers = 8;
// Window half-width scanned for members of a control volume (hop cap).
constexpr int kHopCap = 4;

// Body parameters as seen by device code.
struct BodyDev {
  int kind;
  double cx, cy, cz;
  double a, b, c;
  double theta;
  double ct, st;     // cos and sin of theta (3D vane), evaluated once on the host
  double t_wall;
};

// A box of cells [i0, i0+ni) x [j0, j0+nj).
struct Box2D {
  int i0, j0, ni, nj;
};

// Geometry tables of a 2D grid, all in the caller's geometry buffer.
struct Geo2D;
struct Geo2D {
  int nx, ny, ncell, N, nvel;
  double x0, y0, dx, dy;
  double* phi;       // (nx+1)*(ny+1) vertex level set
  int* type;         // CellType
  int* master;       // master cell, -1 for solid
  int* kind;         // CellKind
  int* flags;        // bit0: centre in gas (eq. ii); bit1: two boundary pieces
  double* lxm; double* lxp; double* lym; double* lyp;
  double* lw; double* nwx; double* nwy; double* rwx; double* rwy;
  double* sbar; double* scv;
  int* irr;          // irregular masters, ascending cell index
  int* mptr;         // CSR pointers (n_irr + 1) into mem
  int* mem;          // members of each irregular master, ascending
  int* counts;       // [0] n_irr, [1] n_members, [2] n_solid, [3] error bits
  double* vnode;     // N velocity nodes
  double2* ghost;    // nvel farfield values (f, g)
  double* wden;      // per irregular-list slot and member: wall-density denominator
  int* aux;          // per cell: scratch of the list builder (member counts, then fill cursors)
};

// Sorts a list of at most kMaxMembers distinct cell indices in place into
// ascending order, each value written at its rank (longer lists, which the
// geometry checks reject, are left as they are).
__device__ inline void sort_cells(int* a, int n) {
  if (n < 2 || n > kMaxMembers) return;
  int v[kMaxMembers];
#pragma unroll
  for (int e = 0; e < kMaxMembers; ++e) v[e] = e < n ? a[e] : 0x7fffffff;
#pragma unroll
  for (int e = 0; e < kMaxMembers; ++e) {
    int r = 0;
#pragma unroll
    for (int f = 0; f < kMaxMembers; ++f) r += v[f] < v[e];
    if (e < n) a[r] = v[e];
  }
}

// consecutive cells per thread and round in the single-block list builders
constexpr int kScanPer = 4;

// Exclusive prefix sum of one int per thread over the block (a multiple of
// 64 threads, at most 1024): a shuffle scan inside each wave, then the wave
// totals through sh (16 ints), two barriers in all.  *total receives the
// block's sum; sh may be reused as soon as the call returns.
__device__ inline int block_scan_excl(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  int before = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    const int sw = sh[w];
    before += w < wave ? sw : 0;
    tot += sw;
  }
  __syncthreads();
  *total = tot;
  return before + x - v;
}

// Cross-lane steps of wave reductions without the LDS crossbar.
// pl32_sum(a, b): lanes 0-31 get a(l) + a(l + 32), lanes 32-63 get
// b(l - 32) + b(l), from one swap of the upper half of a with the lower half
// of b per dword (v_permlane32_swap).  pl16_sum does the same within each
// 32-lane half with 16-lane rows (odd rows of a with even rows of b).
__device__ inline double pl32_sum(double a, double b) {
  const long long ia = __double_as_longlong(a), ib = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap((int)ia, (int)ib, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((int)(ia >> 32), (int)(ib >> 32), false, false);
  const double an = __longlong_as_double(((long long)hi[0] << 32) | (unsigned)lo[0]);
  const double bn = __longlong_as_double(((long long)hi[1] << 32) | (unsigned)lo[1]);
  return an + bn;
}

__device__ inline double pl16_sum(double a, double b) {
  const long long ia = __double_as_longlong(a), ib = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane16_swap((int)ia, (int)ib, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((int)(ia >> 32), (int)(ib >> 32), false, false);
  const double an = __longlong_as_double(((long long)hi[0] << 32) | (unsigned)lo[0]);
  const double bn = __longlong_as_double(((long long)hi[1] << 32) | (unsigned)lo[1]);
  return an + bn;
}

// value of a partner lane inside a 16-lane row (DPP): kMirror16 pairs lane
// i with 15 - i, kMirror8 i with 7 - i in each half row, kSwap2 / kSwap1
// i with i ^ 2 / i ^ 1 in each quad
constexpr int kMirror16 = 0x140, kMirror8 = 0x141, kSwap2 = 0x4E, kSwap1 = 0xB1;
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  // every lane reads a lane of its own row, so no old value is needed
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wave (every lane active); every lane gets the
// same bits, since each step adds the same two operands in both partners.
__device__ inline double wave_allsum(double v) {
  v = pl32_sum(v, v);
  v = pl16_sum(v, v);
  v += dpp_d<kMirror16>(v);
  v += dpp_d<kMirror8>(v);
  v += dpp_d<kSwap2>(v);
  v += dpp_d<kSwap1>(v);
  return v;
}

// an int that other threads update with atomics, read at L2
__device__ inline int load_l2(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One hop of the master search (algorithm (fusion), Appendix A.3) from cell
// (i, j): across the largest gas edge shared with a cell of the domain, ties
// (lengths within 1e-12 of the largest) broken in the order x+, x-, y+, y-.
// Returns false when no edge qualifies.
__device__ inline bool hop2d(const Geo2D& G, int& i, int& j) {
  int c = j * G.nx + i;
  double r = i + 1 < G.nx ? G.lxp[c] : 0.0;
  double l = i > 0 ? G.lxm[c] : 0.0;
  double t = j + 1 < G.ny ? G.lyp[c] : 0.0;
  double b = j > 0 ? G.lym[c] : 0.0;
  double M = fmax(fmax(r, l), fmax(t, b));
  if (!(M > 0.0)) return false;
  double tie = M * (1.0 - 1e-12);
  if (r >= tie) i += 1;
  else if (l >= tie) i -= 1;
  else if (t >= tie) j += 1;
  else j -= 1;
  return true;
}

struct Geo3D {
  int nx, ny, nz, ncell, N, nvel;
  double x0, y0, z0, dx, dy, dz;
  double* phi;       // (nx+1)*(ny+1)*(nz+1)
  int* type; int* master; int* kind; int* flags;
  double* sxm; double* sxp; double* sym; double* syp; double* szm; double* szp;
  double* aw; double* nwx; double* nwy; double* nwz; double* rwx; double* rwy; double* rwz;
  double* vbar; double* vcv;
  int* irr; int* mptr; int* mem; int* counts;
  double* vnode;
  double* ghost;     // nvel farfield values (F)
};

// Scratch of the octree builder, kept with a mesh so that a rebuild into it
// reuses the allocations.
struct AmrBuildScratch {
  std::vector<std::pair<uint64_t, int>> corder;     // coarse cells in Z-order
  std::vector<std::vector<int>> part;               // leaves (depth, i, j, k) per chunk of coarse cells
  std::vector<std::vector<int>> fnb, fdir;          // face entries per chunk of leaves
  std::vector<std::vector<double>> farea;
  std::vector<int> chunk_faces;                     // entries used in each chunk's lists
  std::vector<int> counts;                          // per chunk: irregular CVs, members, solid leaves
};

// Octree mesh (3D): built on the host when the context is created
// (octree3d.hip), uploaded to the geometry buffer when it is bound.  With a
// turning body the host plans every step on the mesh of t^n, then rebuilds
// the mesh for t^{n+1} and the map that carries the state over.
struct AmrHost {
  int n0[3];
  double hf[3];                     // finest spacing
  int nleaf = 0, nface = 0, n_irr = 0, n_members = 0, n_solid = 0;
  std::vector<int> lvl, ijk, type, flags, master;
  std::vector<double> S6, aw, nw, rw, vbar, vcv;
  std::vector<int> fptr, fnb, fdir;  // per leaf, faces x-, x+, y-, y+, z-, z+ (leaf across or -1)
  std::vector<double> farea;
  std::vector<int> cv, cvptr, cvmem; // control volumes: master leaf, members (CSR); regular first
  int nsimple = 0;                   // simple regular control volumes (one face entry per direction)
  int nreg = 0;                      // regular control volumes (one member, no wall face), simple first
  int nf[3] = {0, 0, 0};             // finest-level cells per axis
  std::vector<int> fine;             // leaf containing each finest-level cell
  std::vector<uint64_t> zkey;        // Z-order key of each leaf's lower corner (ascending)
  // turning body, plan of the step from t^n (this mesh) to t^{n+1}
  std::vector<int> type1;            // leaf types with the body at t^{n+1}
  std::vector<double> vbar1;         // leaf gas volumes at t^{n+1}
  std::vector<int> flags1;           // the rest of the leaves' geometry at t^{n+1}, reused by
  std::vector<double> S61, aw1, nw1, r1;   // the build of the mesh of t^{n+1}
  std::vector<double> vnew;          // per master: its control volume's volume at t^{n+1}
  std::vector<int> rptr, rmem;       // per control volume (cv order): leaves receiving its value
  // capacities of the device arrays (the largest mesh a turning body is expected to need)
  int cap_leaf = 0, cap_face = 0;
  AmrBuildScratch scratch;
};

// State carried from the mesh of t^n to the mesh of t^{n+1}: new leaf q
// takes sum_e wgt[e] F[src[e]] / sum_e wgt[e] over e in [sptr[q], sptr[q+1])
// (0 with no entry).
struct AmrRemap {
  std::vector<int> sptr, src;
  std::vector<double> wgt;
};

struct AmrDev {
  int nleaf, ncv, nreg, nsimple;
  int* type; int* master;
  int* cv; int* cvptr; int* cvmem;
  int* fptr; int* fnb; int* fdir;
  double* farea; double* aw; double* nw; double* vbar; double* vcv;
  double* ghost;                    // nvel farfield values
  // turning body
  double* rw;                       // wall centres (3 per leaf)
  double* vnew;                     // per master: volume at t^{n+1}
  int* rptr; int* rmem;             // receivers per control volume
  int* sptr; int* src; double* wgt; // remap to the next mesh
};

// Scratch layout (caller's scratch buffer).
struct Scratch {
  // moving bodies: per-step dispatch and receiving control volumes
  int* skind;        // per-cell kind of the steps of parity 0
  int* skind2;       // per-cell kind of the steps of parity 1
  int* target;       // per cell: master at t^n of the control volume it receives from, -1 none
  int* rcnt;         // per master: receivers other than itself
  int* age;          // consecutive time levels a cell has been solid (saturates at 2)
  int* gl;           // general control volumes (master) or -1-c (cell to zero)
  int* gptr;         // receivers CSR pointers
  int* gmem;         // receivers
  int* gcount;       // [0] entries in gl, [1] error bits, [2] general control volumes,
                     // [4 + parity] entries of the step of that parity (its mass row)
  double* pose;      // pose at t^{n+1}: cx, cy, theta
  double* mom;       // 2D: ncell * 4 (rho, ux, uy, T); 3D: ncell * 8 (Maxwellian factor, u,
                     // 1/(2T), dt/tau, rho)
  double* part;      // 3D: per cell and velocity chunk, sums of F, v F, |v|^2 F (Shakhov: and
                     // v v^T F, |v|^2 v F)
  double* mom2;      // 2D semi-implicit step: moments of the new state (ncell * 4)
  double* heat;      // Shakhov: heat flux of each cell's control volume (2D: 2, 3D: 3 per cell)
  double* heat2;     // 2D semi-implicit Shakhov step: heat flux of the new state
  double* nu;        // semi-implicit step: dt/tau of each control volume at t^n
  double* fslot;     // 2 x per irregular master: Fx, Fy, torque (2D) / Fx, Fy, Fz (3D)
  double* mpart;     // 2 x mass partials (regular tiles, then control volumes)
  int mpart_cap;
  double* body;      // rigid body state on device: cx, cy, theta, ux, uy, omega
  double* red;       // small reduction buffer
};

// Per-kernel HIP events recorded around every launch while profiling is on;
// elapsed times are summed when read.
constexpr int kProfKernels = 6;
constexpr int kProfCap = 4096;
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> start[kProfKernels], stop[kProfKernels];
  int count[kProfKernels] = {0, 0, 0, 0, 0, 0};
  double host_ms[3] = {0.0, 0.0, 0.0};   // turning body: planning, launch to remap map, mesh build
  int host_count[3] = {0, 0, 0};
};

}  // namespace ccdvm

struct cc_ctx {
  cc_config cfg;
  cc_body body;
  int dim;
  int nx, ny, nz, ncell, N, nvel;
  double dx, dy, dz, dv, dt;
  double vmax_abs;
  size_t state_bytes, geom_bytes, scratch_bytes;
  void* state[2] = {nullptr, nullptr};
  int cur = 0;
  void* geom = nullptr;
  void* scratch = nullptr;
  int static_dev = -1;     // device whose static scratch array this context is bound to (-1: none)
  bool scratch_taken = false;  // another context was bound to that array since
  double cfl[2] = {0.0, 0.0};  // positivity number of eq. eq-CFL: transport, collisions
  bool bound_geometry = false;  // a uniform grid's geometry has been built on the device
  hipStream_t stream = nullptr;
  bool bound = false;
  bool merged = false;     // members hold their control-volume value
  bool mom_valid = false;  // scratch.mom holds the moments of the current state
  int step_parity = 0;     // which half of the double-buffered partials the next step writes
  int last_args_ntiles = 0;
  int seglen = 0;          // rows per regular-cell tile (0: automatic)
  ccdvm::Geo2D g2;          // geometry at the current time
  ccdvm::Geo2D g2n;         // moving bodies: geometry at the next time level
  long long nstep = 0;      // steps taken since binding
  ccdvm::Geo3D g3;
  bool amr = false;                 // 3D octree mesh
  bool amr_turning = false;         // octree with a body turning about the z axis
  bool amr_leaf_records = false;    // the remap wrote every leaf's record: only control
                                    // volumes with several members need merge and moments
  ccdvm::AmrHost* amrh = nullptr;
  ccdvm::AmrHost* amr_spare = nullptr;   // turning body: the previous mesh, rebuilt into next step
  ccdvm::AmrDev a3{};
  hipStream_t side = nullptr;        // octree: cut control volumes run beside the others
  hipEvent_t fork = nullptr, join = nullptr;
  ccdvm::Scratch s;
  int n_irr = 0, n_members = 0, n_solid = 0;
  // host mirror of the rigid body (kept in sync with the device copy)
  double body_state[6] = {0, 0, 0, 0, 0, 0};
  ccdvm::Prof prof;
  std::string err;
};

struct cc_batch {
  std::vector<cc_ctx*> ctx;
  std::vector<int> base_cur;        // each instance's current buffer when the tables were built
  hipStream_t stream = nullptr;
  char* dev = nullptr;              // caller-owned workspace
  size_t dev_bytes = 0;
  void* d_desc0 = nullptr;
  void* d_desc1 = nullptr;
  int2* d_tiles = nullptr;
  int2* d_cuts = nullptr;
  size_t tile_cap = 0, cut_cap = 0;
  int ncut = 0;
  std::vector<int> group_nch, group_rows, group_off, group_cnt;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  long long steps = 0;              // batched steps since the tables were built
  bool bound = false;
  std::string err;
};

namespace ccdvm {

// batched step (step2d.hip)
int batch_group_nch(const cc_ctx* ctx);
bool batch_supported_nch(int nch);
size_t batch_desc_bytes();
void batch_fill(cc_batch* B, std::vector<char>& desc0, std::vector<char>& desc1,
                std::vector<int2>& tiles, std::vector<int2>& cuts);
hipError_t batch_launch_step(cc_batch* B, int par, hipStream_t* side, int nside);
hipError_t batch_launch_desc(cc_batch* B, const void* D, hipStream_t* side, int nside);
void batch_desc_patch(void* desc, const double2* in, double2* out, double* mom);
// batched adjoint (adjoint2d.hip)
size_t batch_adjoint_workspace_bytes(const cc_batch* B, int nsteps, int K);
hipError_t batch_adjoint_run_2d(cc_batch* B, int nsteps, int K, int objective, char* ws, double* out);
hipError_t batch_launch_group(cc_batch* B, int g);
int tile_rows(const cc_ctx* ctx);

// geometry (geom2d.hip / geom3d.hip)
hipError_t build_geometry_2d(cc_ctx* ctx, Geo2D& G, const double* pose);
hipError_t build_geometry_box_2d(cc_ctx* ctx, Geo2D& G, const double* pose, Box2D bx);
hipError_t build_geometry_3d(cc_ctx* ctx);
// largest outflow rate per unit area (volume) of the cut and merged control
// volumes, eq. phiCFL (geom2d.hip / geom3d.hip); synchronise the stream
hipError_t cfl_rate_2d(cc_ctx* ctx, double vlo, double vhi, const double* body_state, double* rate);
hipError_t cfl_rate_3d(cc_ctx* ctx, double vlo, double vhi, double* rate);

// step and helpers (step2d.hip / step3d.hip)
hipError_t launch_init_maxwellian_2d(cc_ctx* ctx);
hipError_t launch_load_state_2d(cc_ctx* ctx, const double* f, const double* g);
hipError_t launch_store_state_2d(const cc_ctx* ctx, double* f, double* g);
hipError_t launch_merge_2d(cc_ctx* ctx);
// moments of every gas cell, or (regular_only) of the regular cells only
hipError_t launch_moments_all_2d(cc_ctx* ctx, bool regular_only = false);
hipError_t launch_step_2d_fused(cc_ctx* ctx, bool reduce_prev, double* prev_force_row,
                                double* cur_mass_row, bool record, bool relax = true,
                                bool implicit = false);
hipError_t launch_step_2d_flush(cc_ctx* ctx, double* force_row, double* mass_row);
hipError_t launch_mass_2d(cc_ctx* ctx, double* mass_row);
hipError_t launch_moments_out_2d(cc_ctx* ctx, double* out);

hipError_t launch_init_maxwellian_3d(cc_ctx* ctx);
hipError_t launch_load_state_3d(cc_ctx* ctx, const double* f);
hipError_t launch_store_state_3d(const cc_ctx* ctx, double* f);
hipError_t launch_merge_3d(cc_ctx* ctx);
hipError_t launch_moments_all_3d(cc_ctx* ctx);
hipError_t launch_step_3d(cc_ctx* ctx, double* force_row, double* mass_row);
hipError_t launch_mass_3d(cc_ctx* ctx, double* mass_row);
hipError_t launch_moments_out_3d(cc_ctx* ctx, double* out);
int chunks3d(int N);   // velocity chunks of the 3D regular-cell pass (0: unsupported N)

// octree mesh (octree3d.hip)
// prev (nullable): a mesh whose plan holds the geometry of its leaves at the
// same angle, reused for the leaves both meshes share
bool build_octree_3d(const cc_config& cfg, const cc_body& body, double theta, AmrHost& H, std::string& err,
                     const AmrHost* prev = nullptr);
bool plan_amr_move(const cc_config& cfg, const cc_body& body, double th1, AmrHost& H, std::string& err);
void build_amr_remap(const AmrHost& old_mesh, const AmrHost& new_mesh, int depth, AmrRemap& R);
hipError_t launch_amr_remap(cc_ctx* ctx, const double* from, double* to);
hipError_t launch_amr_tables(cc_ctx* ctx);
hipError_t launch_amr_init(cc_ctx* ctx, const double* f);   // f null: farfield Maxwellian
// from: first control volume (the others are single members whose
// records are already valid)
hipError_t launch_amr_merge(cc_ctx* ctx, int from = 0);
hipError_t launch_amr_moments(cc_ctx* ctx, int from = 0);
hipError_t launch_amr_step(cc_ctx* ctx, double* row);

// profiling hooks (capi.cpp)
void prof_begin(cc_ctx* ctx, int k);
void prof_end(cc_ctx* ctx, int k);

}  // namespace ccdvm
