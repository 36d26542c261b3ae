// C-ABI of the ccdvm library: validation, buffer layout, orchestration of the
// device kernels on the caller's stream.  The declarations and their
// contracts are in include/ccdvm.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <future>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ccdvm_impl.h"

using namespace ccdvm;

namespace ccdvm {
bool regular_supported_2d(int nvel);
bool regular_supported_3d(int nvel);
hipError_t launch_force_only_2d(cc_ctx* ctx, double* out4);
hipError_t launch_force_only_3d(cc_ctx* ctx, double* out4);
hipError_t launch_moving_prologue_2d(cc_ctx* ctx);
hipError_t launch_moving_step_2d(cc_ctx* ctx, double* force_row, double* mass_row, bool next);
hipError_t launch_moving_init_2d(cc_ctx* ctx);
size_t adjoint_workspace_bytes(const cc_ctx* ctx, int nsteps, int K);
hipError_t adjoint_run_2d(cc_ctx* ctx, int nsteps, int K, int objective, char* pool, double* out);
hipError_t launch_imex_step_2d(cc_ctx* ctx, double* row);
bool imex_fused_2d(const cc_ctx* ctx);
hipError_t launch_imex_fused_2d(cc_ctx* ctx, bool reduce_prev, double* prev_force_row, double* cur_mass_row);
}  // namespace ccdvm

static bool is_moving(const cc_ctx* ctx) {
  return ctx->body.motion != CC_MOTION_FIXED && ctx->body.kind != CC_BODY_NONE;
}

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Bump allocator over a caller buffer; with base == nullptr it only sizes.
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

void layout_geo2d_one(cc_ctx* ctx, Geo2D& G, char* base, size_t* bytes) {
  Carver cv{base};
  G.nx = ctx->nx; G.ny = ctx->ny; G.ncell = ctx->ncell; G.N = ctx->N; G.nvel = ctx->nvel;
  G.x0 = ctx->cfg.lo[0]; G.y0 = ctx->cfg.lo[1]; G.dx = ctx->dx; G.dy = ctx->dy;
  size_t n = ctx->ncell;
  G.phi = cv.take<double>((size_t)(ctx->nx + 1) * (ctx->ny + 1));
  G.type = cv.take<int>(n); G.master = cv.take<int>(n); G.kind = cv.take<int>(n);
  G.flags = cv.take<int>(n);
  G.lxm = cv.take<double>(n); G.lxp = cv.take<double>(n);
  G.lym = cv.take<double>(n); G.lyp = cv.take<double>(n);
  G.lw = cv.take<double>(n); G.nwx = cv.take<double>(n); G.nwy = cv.take<double>(n);
  G.rwx = cv.take<double>(n); G.rwy = cv.take<double>(n);
  G.sbar = cv.take<double>(n); G.scv = cv.take<double>(n);
  G.irr = cv.take<int>(n); G.mptr = cv.take<int>(n + 1); G.mem = cv.take<int>(n);
  G.aux = cv.take<int>(n);
  G.counts = cv.take<int>(4);
  G.vnode = cv.take<double>(ctx->N);
  G.ghost = cv.take<double2>(ctx->nvel);
  G.wden = nullptr;
  *bytes = cv.off;
}

// one geometry level for a fixed body, two (t^n, t^{n+1}) for a moving one
void layout_geo2d(cc_ctx* ctx, char* base, size_t* bytes) {
  size_t one = 0;
  layout_geo2d_one(ctx, ctx->g2, base, &one);
  *bytes = one;
  if (is_moving(ctx)) {
    layout_geo2d_one(ctx, ctx->g2n, base ? base + one : nullptr, &one);
    *bytes = 2 * one;
  }
}

void layout_geo3d(cc_ctx* ctx, char* base, size_t* bytes) {
  Carver cv{base};
  Geo3D& G = ctx->g3;
  G.nx = ctx->nx; G.ny = ctx->ny; G.nz = ctx->nz; G.ncell = ctx->ncell; G.N = ctx->N;
  G.nvel = ctx->nvel;
  G.x0 = ctx->cfg.lo[0]; G.y0 = ctx->cfg.lo[1]; G.z0 = ctx->cfg.lo[2];
  G.dx = ctx->dx; G.dy = ctx->dy; G.dz = ctx->dz;
  size_t n = ctx->ncell;
  G.phi = cv.take<double>((size_t)(ctx->nx + 1) * (ctx->ny + 1) * (ctx->nz + 1));
  G.type = cv.take<int>(n); G.master = cv.take<int>(n); G.kind = cv.take<int>(n);
  G.flags = cv.take<int>(n);
  G.sxm = cv.take<double>(n); G.sxp = cv.take<double>(n); G.sym = cv.take<double>(n);
  G.syp = cv.take<double>(n); G.szm = cv.take<double>(n); G.szp = cv.take<double>(n);
  G.aw = cv.take<double>(n); G.nwx = cv.take<double>(n); G.nwy = cv.take<double>(n);
  G.nwz = cv.take<double>(n); G.rwx = cv.take<double>(n); G.rwy = cv.take<double>(n);
  G.rwz = cv.take<double>(n);
  G.vbar = cv.take<double>(n); G.vcv = cv.take<double>(n);
  G.irr = cv.take<int>(n); G.mptr = cv.take<int>(n + 1); G.mem = cv.take<int>(n);
  G.counts = cv.take<int>(4);
  G.vnode = cv.take<double>(ctx->N);
  G.ghost = cv.take<double>(ctx->nvel);
  *bytes = cv.off;
}

// leaves the buffers are sized for: the mesh, or with a turning body the
// largest mesh expected
size_t cell_capacity(const cc_ctx* ctx) {
  return ctx->amr_turning ? (size_t)ctx->amrh->cap_leaf : (size_t)ctx->ncell;
}

void layout_amr(cc_ctx* ctx, char* base, size_t* bytes) {
  Carver cv{base};
  const AmrHost& H = *ctx->amrh;
  AmrDev& G = ctx->a3;
  const bool turn = ctx->amr_turning;
  const size_t n = turn ? H.cap_leaf : H.nleaf, nf = turn ? H.cap_face : H.nface;
  const size_t ncv = turn ? n : H.cv.size(), nmem = turn ? n : H.cvmem.size();
  G.nleaf = H.nleaf; G.ncv = (int)H.cv.size(); G.nreg = H.nreg; G.nsimple = H.nsimple;
  G.type = cv.take<int>(n); G.master = cv.take<int>(n);
  G.cv = cv.take<int>(ncv); G.cvptr = cv.take<int>(ncv + 1); G.cvmem = cv.take<int>(nmem);
  G.fptr = cv.take<int>(n + 1); G.fnb = cv.take<int>(nf); G.fdir = cv.take<int>(nf);
  G.farea = cv.take<double>(nf); G.aw = cv.take<double>(n); G.nw = cv.take<double>(3 * n);
  G.vbar = cv.take<double>(n); G.vcv = cv.take<double>(n);
  G.ghost = cv.take<double>(ctx->nvel);
  G.rw = turn ? cv.take<double>(3 * n) : nullptr;
  G.vnew = turn ? cv.take<double>(n) : nullptr;
  G.rptr = turn ? cv.take<int>(n + 1) : nullptr;
  G.rmem = turn ? cv.take<int>(n) : nullptr;
  G.sptr = turn ? cv.take<int>(n + 1) : nullptr;
  G.src = turn ? cv.take<int>(2 * n) : nullptr;
  G.wgt = turn ? cv.take<double>(2 * n) : nullptr;
  *bytes = cv.off;
}

void layout_scratch(cc_ctx* ctx, char* base, size_t* bytes) {
  Carver cv{base};
  size_t n = cell_capacity(ctx);
  int nm = ctx->dim == 2 ? 4 : 8;
  ctx->s.skind = cv.take<int>(n);
  ctx->s.skind2 = cv.take<int>(n);
  ctx->s.target = cv.take<int>(n);
  ctx->s.rcnt = cv.take<int>(n);
  ctx->s.age = cv.take<int>(n);
  ctx->s.gl = cv.take<int>(n);
  ctx->s.gptr = cv.take<int>(n + 1);
  ctx->s.gmem = cv.take<int>(n);
  ctx->s.gcount = cv.take<int>(8);
  ctx->s.pose = cv.take<double>(4);
  ctx->s.mom = cv.take<double>(n * nm);
  ctx->s.mom2 = cv.take<double>(ctx->dim == 2 ? n * 4 : 0);
  const bool sk = ctx->cfg.model == CC_MODEL_SHAKHOV;
  ctx->s.heat = sk ? cv.take<double>(n * (ctx->dim == 2 ? 2 : 3)) : nullptr;
  ctx->s.heat2 = sk && ctx->dim == 2 ? cv.take<double>(n * 2) : nullptr;
  ctx->s.nu = cv.take<double>(n);
  // 3D chunk sums: 5 per chunk, 14 with the Shakhov model (second and third moments)
  const size_t nsum = ctx->cfg.model == CC_MODEL_SHAKHOV ? 14 : 5;
  ctx->s.part = ctx->dim == 3 ? cv.take<double>(n * (size_t)chunks3d(ctx->N) * nsum) : nullptr;
  ctx->s.fslot = cv.take<double>(n * 3 * 2);
  ctx->s.mpart_cap = (int)((size_t)((ctx->nx + 3) / 4) * ctx->ny * ctx->nz + n);
  ctx->s.mpart = cv.take<double>((size_t)ctx->s.mpart_cap * 2);
  ctx->s.body = cv.take<double>(16);
  ctx->s.red = cv.take<double>(4 * 128 + 8);
  *bytes = cv.off;
}

cc_status fail(cc_ctx* ctx, cc_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

cc_status not_bound(cc_ctx* ctx) {
  return fail(ctx, CC_ESTATE, ctx->scratch_taken
                                  ? "another context was bound to this GPU's static scratch array: bind again"
                                  : "cc_bind first");
}

cc_status hip_fail(cc_ctx* ctx, hipError_t e, const char* where) {
  return fail(ctx, CC_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, expr, where)                      \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
  } while (0)

}  // namespace

namespace ccdvm {

void prof_begin(cc_ctx* ctx, int k) {
  Prof& P = ctx->prof;
  if (!P.on || P.count[k] >= (int)P.start[k].size()) return;
  hipEventRecord(P.start[k][P.count[k]], ctx->stream);
}

void prof_end(cc_ctx* ctx, int k) {
  Prof& P = ctx->prof;
  if (!P.on || P.count[k] >= (int)P.stop[k].size()) return;
  hipEventRecord(P.stop[k][P.count[k]], ctx->stream);
  P.count[k] += 1;
}

}  // namespace ccdvm

namespace {

// Exceptions do not cross the C interface: a host allocation that fails,
// or a host thread that cannot start, ends the call with CC_ENOMEM and the
// reason in the object's last error (when there is an object to hold it).
template <class F>
cc_status no_throw(std::string* err, F&& f) noexcept {
  const char* why = "unexpected host error";
  try {
    return f();
  } catch (const std::bad_alloc&) {
    why = "host allocation failed";
  } catch (const std::exception& e) {
    if (err) {
      try { *err = std::string("host error: ") + e.what(); } catch (...) {}
    }
    return CC_ENOMEM;
  } catch (...) {
  }
  if (err) {
    try { *err = why; } catch (...) {}
  }
  return CC_ENOMEM;
}

// The octree of the initial angle; for a turning body also the capacities
// of the device arrays: the largest mesh over a half turn (16 angles; the
// vane and the sphere map onto themselves after half a turn), plus a margin.
cc_status build_first_mesh(const cc_config& c, const cc_body& body, bool turning, AmrHost& H) {
  std::string err;
  if (!build_octree_3d(c, body, body.theta, H, err)) {
    fprintf(stderr, "ccdvm: %s\n", err.c_str());
    return CC_EGEOM;
  }
  if (!turning) return CC_OK;
  int ml = H.nleaf, mf = H.nface;
  for (int k = 1; k < 16; ++k) {
    AmrHost T;
    if (!build_octree_3d(c, body, body.theta + k * M_PI / 16.0, T, err)) {
      fprintf(stderr, "ccdvm: %s (at a later angle)\n", err.c_str());
      return CC_EGEOM;
    }
    ml = std::max(ml, T.nleaf);
    mf = std::max(mf, T.nface);
  }
  H.cap_leaf = ml + ml / 4 + 64;
  H.cap_face = mf + mf / 4 + 256;
  return CC_OK;
}

static cc_status check_cfl(cc_ctx* ctx, bool report);

cc_status create_impl(const cc_config* cfg, const cc_body* body, cc_ctx** out) {
  if (!cfg || !body || !out) return CC_EINVAL;
  *out = nullptr;
  cc_ctx* ctx = new (std::nothrow) cc_ctx();
  if (!ctx) return CC_ENOMEM;
  ctx->cfg = *cfg;
  ctx->body = *body;
  const cc_config& c = *cfg;
  auto reject = [&](const char* msg) {
    fprintf(stderr, "ccdvm: %s\n", msg);
    delete ctx;
    return CC_EINVAL;
  };
  if (c.dim != 2 && c.dim != 3) return reject("dim must be 2 or 3");
  for (int d = 0; d < c.dim; ++d) {
    if (c.n[d] < 1) return reject("grid size must be >= 1");
    if (!(c.hi[d] > c.lo[d])) return reject("empty domain");
  }
  if (c.dim == 2 && c.n[2] != 1) return reject("n[2] must be 1 in 2D");
  if (c.nv < 1 || c.nv > 64) return reject("nv must be in [1, 64]");
  if (!(c.vmax > c.vmin)) return reject("empty velocity box");
  if (!(c.cfl > 0.0) && !(c.dt > 0.0)) return reject("need cfl > 0 or dt > 0");
  if (!(c.inflow[0] > 0.0) || !(c.inflow[4] > 0.0)) return reject("inflow rho and T must be > 0");
  if (c.kn > 0.0 && !(c.lref > 0.0)) return reject("lref must be > 0");
  if (body->kind < CC_BODY_NONE || body->kind > CC_BODY_VANE) return reject("unknown body kind");
  if (c.dim == 2 && (body->kind == CC_BODY_SPHERE || body->kind == CC_BODY_VANE))
    return reject("sphere and vane are 3D only");
  if (c.dim == 3 && body->kind != CC_BODY_SPHERE && body->kind != CC_BODY_VANE && body->kind != CC_BODY_NONE)
    return reject("3D supports a sphere, a vane or no body");
  if (body->kind == CC_BODY_VANE && !(body->axes[0] > 0.0 && body->axes[1] > 0.0 && body->axes[2] > 0.0))
    return reject("vane half-sizes must be > 0");
  if (body->kind != CC_BODY_NONE && !(body->t_wall > 0.0)) return reject("t_wall must be > 0");
  if (body->kind == CC_BODY_ELLIPSE && !(body->axes[0] > 0.0 && body->axes[1] > 0.0))
    return reject("ellipse semi-axes must be > 0");
  if ((body->kind == CC_BODY_CIRCLE || body->kind == CC_BODY_CAVITY || body->kind == CC_BODY_SPHERE) &&
      !(body->axes[0] > 0.0))
    return reject("radius must be > 0");
  if (body->motion < CC_MOTION_FIXED || body->motion > CC_MOTION_IMPOSED) return reject("unknown motion");
  // 3D: a body turning about the z axis through its centre (pure rotation)
  const bool turning3 = c.dim == 3 && body->motion != CC_MOTION_FIXED && body->kind != CC_BODY_NONE;
  if (turning3 && (body->vel[0] != 0.0 || body->vel[1] != 0.0 || body->vel[2] != 0.0))
    return reject("a 3D body only turns about the z axis through its centre (vel must be 0)");
  if (c.dim == 2 && body->motion != CC_MOTION_FIXED && body->kind != CC_BODY_CIRCLE &&
      body->kind != CC_BODY_ELLIPSE && body->kind != CC_BODY_NONE)
    return reject("moving bodies must be circles or ellipses");
  if (body->motion == CC_MOTION_FREE_ROTATION && !(body->inertia > 0.0))
    return reject("inertia must be > 0");
  if (c.maxwellian != CC_MAXW_DIRECT && c.maxwellian != CC_MAXW_CONSERVATIVE)
    return reject("unknown maxwellian mode");
  if (c.maxwellian == CC_MAXW_CONSERVATIVE && body->motion != CC_MOTION_FIXED && body->kind != CC_BODY_NONE)
    return reject("the conservative equilibrium is available for fixed bodies");
  if (c.scheme != CC_SCHEME_EXPLICIT && c.scheme != CC_SCHEME_IMEX) return reject("unknown scheme");
  if (c.model != CC_MODEL_BGK && c.model != CC_MODEL_SHAKHOV) return reject("unknown relaxation model");
  if (c.model == CC_MODEL_SHAKHOV && !(c.prandtl > 0.0 && isfinite(c.prandtl)))
    return reject("the Shakhov model needs a finite Prandtl number > 0");
  if (c.scheme == CC_SCHEME_IMEX && body->motion != CC_MOTION_FIXED && body->kind != CC_BODY_NONE)
    return reject("the semi-implicit scheme is available for fixed bodies");
  if (c.amr_depth < 0 || c.amr_depth > 8) return reject("amr_depth must be in [0, 8]");
  if (c.amr_depth > 0 || turning3) {
    if (c.dim != 3) return reject("the octree mesh is 3D");
    for (int d = 0; d < 3; ++d)
      if (((long long)c.n[d] << c.amr_depth) >= (1LL << 20)) return reject("octree too deep for the coarse grid");
    if (c.model != CC_MODEL_BGK || c.maxwellian != CC_MAXW_DIRECT || c.scheme != CC_SCHEME_EXPLICIT)
      return reject("the octree mesh runs the explicit BGK scheme with the direct equilibrium");
  }
  ctx->dim = c.dim;
  ctx->nx = c.n[0]; ctx->ny = c.n[1]; ctx->nz = c.dim == 3 ? c.n[2] : 1;
  long long ncell = (long long)ctx->nx * ctx->ny * ctx->nz;
  if (ncell > (1LL << 30)) return reject("too many cells");
  ctx->ncell = (int)ncell;
  ctx->N = c.nv;
  ctx->nvel = c.dim == 2 ? c.nv * c.nv : c.nv * c.nv * c.nv;
  if (c.dim == 2 && !regular_supported_2d(ctx->nvel)) return reject("unsupported velocity grid size");
  if (c.dim == 3 && !regular_supported_3d(ctx->nvel))
    return reject("unsupported velocity grid size (3D: N in {4, 6, 8, 12, 16})");
  if (c.dim == 3 && fabs(c.vmin + c.vmax) > 1e-12 * fabs(c.vmax))
    return reject("3D needs a velocity box symmetric about 0");
  ctx->dx = (c.hi[0] - c.lo[0]) / ctx->nx;
  ctx->dy = (c.hi[1] - c.lo[1]) / ctx->ny;
  ctx->dz = c.dim == 3 ? (c.hi[2] - c.lo[2]) / ctx->nz : 1.0;
  if (c.amr_depth > 0 || turning3) {
    // octree mesh (a turning body always runs on it; depth 0 is the uniform grid)
    ctx->amr = true;
    ctx->amr_turning = turning3;
    ctx->amrh = new (std::nothrow) AmrHost();
    if (!ctx->amrh) { delete ctx; return CC_ENOMEM; }
    const cc_status st = no_throw(nullptr, [&] { return build_first_mesh(c, *body, turning3, *ctx->amrh); });
    if (st != CC_OK) {
      if (st == CC_ENOMEM) fprintf(stderr, "ccdvm: host allocation failed while building the octree\n");
      delete ctx->amrh;
      delete ctx;
      return st;
    }
    // the leaves are the cells; the finest spacing sets dt
    ctx->ncell = ctx->amrh->nleaf;
    ctx->dx = ctx->amrh->hf[0]; ctx->dy = ctx->amrh->hf[1]; ctx->dz = ctx->amrh->hf[2];
  }
  ctx->dv = (c.vmax - c.vmin) / c.nv;
  double vm = 0.0;
  for (int p = 0; p < c.nv; ++p) vm = fmax(vm, fabs(c.vmin + (p + 0.5) * ctx->dv));
  ctx->vmax_abs = vm;
  // dt = CFL / sum_d max|v_d| / dx_d (simple form of the positivity condition)
  double rate = vm / ctx->dx + vm / ctx->dy + (c.dim == 3 ? vm / ctx->dz : 0.0);
  ctx->dt = c.dt > 0.0 ? c.dt : c.cfl / rate;
  size_t per = c.dim == 2 ? 16 : 8;
  ctx->state_bytes = align_up(cell_capacity(ctx) * ctx->nvel * per);
  if (c.dim == 2) layout_geo2d(ctx, nullptr, &ctx->geom_bytes);
  else if (ctx->amr) layout_amr(ctx, nullptr, &ctx->geom_bytes);
  else layout_geo3d(ctx, nullptr, &ctx->geom_bytes);
  layout_scratch(ctx, nullptr, &ctx->scratch_bytes);
  ctx->body_state[0] = body->center[0];
  ctx->body_state[1] = body->center[1];
  ctx->body_state[2] = body->theta;
  if (body->motion != CC_MOTION_FIXED) {
    ctx->body_state[3] = body->vel[0];
    ctx->body_state[4] = body->vel[1];
    ctx->body_state[5] = body->omega;
  }
  // the octree is built on the host: its positivity number is known now
  if (ctx->amr) check_cfl(ctx, false);
  *out = ctx;
  return CC_OK;
}

cc_status workspace_bytes_impl(const cc_ctx* ctx, size_t* state_bytes, size_t* geom_bytes,
                               size_t* scratch_bytes) {
  if (!ctx) return CC_EINVAL;
  if (state_bytes) *state_bytes = ctx->state_bytes;
  if (geom_bytes) *geom_bytes = ctx->geom_bytes;
  if (scratch_bytes) *scratch_bytes = ctx->scratch_bytes;
  return CC_OK;
}

cc_status dt_impl(const cc_ctx* ctx, double* dt) {
  if (!ctx || !dt) return CC_EINVAL;
  *dt = ctx->dt;
  return CC_OK;
}

// host mesh -> device arrays (the host vectors stay unchanged until the
// stream has been synchronised)
static hipError_t upload_amr_mesh(cc_ctx* ctx) {
  const AmrHost& H = *ctx->amrh;
  AmrDev& G = ctx->a3;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream) : hipSuccess;
  };
  const size_t n = H.nleaf;
  G.nleaf = H.nleaf; G.ncv = (int)H.cv.size(); G.nreg = H.nreg; G.nsimple = H.nsimple;
  hipError_t e = hipSuccess;
  for (hipError_t x : {up(G.type, H.type.data(), n * sizeof(int)), up(G.master, H.master.data(), n * sizeof(int)),
                       up(G.cv, H.cv.data(), H.cv.size() * sizeof(int)),
                       up(G.cvptr, H.cvptr.data(), H.cvptr.size() * sizeof(int)),
                       up(G.cvmem, H.cvmem.data(), H.cvmem.size() * sizeof(int)),
                       up(G.fptr, H.fptr.data(), H.fptr.size() * sizeof(int)),
                       up(G.fnb, H.fnb.data(), H.fnb.size() * sizeof(int)),
                       up(G.fdir, H.fdir.data(), H.fdir.size() * sizeof(int)),
                       up(G.farea, H.farea.data(), H.farea.size() * sizeof(double)),
                       up(G.aw, H.aw.data(), n * sizeof(double)), up(G.nw, H.nw.data(), 3 * n * sizeof(double)),
                       up(G.vbar, H.vbar.data(), n * sizeof(double)), up(G.vcv, H.vcv.data(), n * sizeof(double)),
                       G.rw ? up(G.rw, H.rw.data(), 3 * n * sizeof(double)) : hipSuccess})
    if (x != hipSuccess) e = x;
  ctx->g3.ncell = H.nleaf;
  return e;
}

// the control volumes in this step's order, their volumes at t^{n+1} and
// their receivers (turning body)
static hipError_t upload_amr_plan(cc_ctx* ctx) {
  const AmrHost& H = *ctx->amrh;
  AmrDev& G = ctx->a3;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream) : hipSuccess;
  };
  G.ncv = (int)H.cv.size(); G.nreg = H.nreg; G.nsimple = H.nsimple;
  hipError_t e = hipSuccess;
  for (hipError_t x : {up(G.cv, H.cv.data(), H.cv.size() * sizeof(int)),
                       up(G.cvptr, H.cvptr.data(), H.cvptr.size() * sizeof(int)),
                       up(G.cvmem, H.cvmem.data(), H.cvmem.size() * sizeof(int)),
                       up(G.vnew, H.vnew.data(), H.vnew.size() * sizeof(double)),
                       up(G.rptr, H.rptr.data(), H.rptr.size() * sizeof(int)),
                       up(G.rmem, H.rmem.data(), H.rmem.size() * sizeof(int))})
    if (x != hipSuccess) e = x;
  return e;
}

// Outflow rate per unit volume of eq. (phiCFL) over the control volumes of
// an octree mesh (members' face entries, the farfield included, and wall
// faces), maximised over the eight corner nodes of the velocity grid (phi is
// convex in v).  A turning body's walls move with omega e_z x (r - centre).
static double cfl_rate_amr(const AmrHost& H, double vlo, double vhi, double omega, const double* centre) {
  double best = 0.0;
  const int ncv = (int)H.cv.size();
  for (int q = 0; q < ncv; ++q) {
    const int m = H.cv[q];
    for (int corner = 0; corner < 8; ++corner) {
      const double v[3] = {(corner & 1) ? vhi : vlo, (corner & 2) ? vhi : vlo, (corner & 4) ? vhi : vlo};
      double phi = 0.0;
      for (int e = H.cvptr[q]; e < H.cvptr[q + 1]; ++e) {
        const int k = H.cvmem[e];
        for (int f = H.fptr[k]; f < H.fptr[k + 1]; ++f) {
          const int d = H.fdir[f];
          const double vn = (d & 1) ? v[d >> 1] : -v[d >> 1];
          phi += H.farea[f] * fmax(vn, 0.0);
        }
        if (H.aw[k] > 0.0) {
          const double* n = &H.nw[3 * (size_t)k];
          double uwx = 0.0, uwy = 0.0;
          if (omega != 0.0) {
            const double* r = &H.rw[3 * (size_t)k];
            uwx = -omega * (r[1] - centre[1]);
            uwy = omega * (r[0] - centre[0]);
          }
          phi += H.aw[k] * fmax((v[0] - uwx) * n[0] + (v[1] - uwy) * n[1] + v[2] * n[2], 0.0);
        }
      }
      best = fmax(best, phi / H.vcv[m]);
    }
  }
  return best;
}

// Positivity number of eq. (eq-CFL) on the bound geometry: dt times the
// largest outflow rate per unit area (volume) of a control volume, and dt
// times the largest collision frequency 1/tau at the inflow density
// (explicit scheme only).  Regular cells: phi / S = sum_d |v_d| / dx_d,
// largest at the grid's extreme nodes.  Warns above 1, or fails with
// CC_ECFL when cfl_strict is set.
static cc_status check_cfl(cc_ctx* ctx, bool report) {
  const cc_config& c = ctx->cfg;
  const double vlo = c.vmin + 0.5 * ctx->dv, vhi = c.vmin + (c.nv - 0.5) * ctx->dv;
  const double vm = ctx->vmax_abs;
  double rate = 0.0;
  if (ctx->amr) {
    rate = cfl_rate_amr(*ctx->amrh, vlo, vhi, ctx->amr_turning ? ctx->body_state[5] : 0.0, ctx->body.center);
  } else if (!ctx->bound_geometry) {
    return CC_OK;   // uniform grids: the geometry is built on the device by cc_bind
  } else {
    rate = vm / ctx->dx + vm / ctx->dy + (ctx->dim == 3 ? vm / ctx->dz : 0.0);
    double irr = 0.0;
    const hipError_t e = ctx->dim == 2 ? cfl_rate_2d(ctx, vlo, vhi, ctx->body_state, &irr)
                                       : cfl_rate_3d(ctx, vlo, vhi, &irr);
    if (e != hipSuccess) return hip_fail(ctx, e, "positivity check");
    rate = fmax(rate, irr);
  }
  ctx->cfl[0] = ctx->dt * rate;
  const double tau_coef = sqrt(M_PI) / 2.0 * c.kn * c.lref / sqrt(2.0);
  ctx->cfl[1] = c.kn > 0.0 && c.scheme == CC_SCHEME_EXPLICIT ? ctx->dt * c.inflow[0] / tau_coef : 0.0;
  const double num = ctx->cfl[0] + ctx->cfl[1];
  if (report && num > 1.0) {
    char msg[200];
    snprintf(msg, sizeof(msg),
             "positivity condition eq-CFL: dt (max 1/tau + max phi/S) = %.4g > 1 (transport %.4g, collisions %.4g)",
             num, ctx->cfl[0], ctx->cfl[1]);
    if (c.cfl_strict) return fail(ctx, CC_ECFL, msg);
    fprintf(stderr, "ccdvm: warning: %s\n", msg);
  }
  return CC_OK;
}

cc_status cfl_number_impl(const cc_ctx* ctx, double* out) {
  if (!ctx || !out) return CC_EINVAL;
  if (!ctx->bound && !ctx->amr) return CC_ESTATE;
  out[0] = ctx->cfl[0];
  out[1] = ctx->cfl[1];
  out[2] = ctx->cfl[0] + ctx->cfl[1];
  return CC_OK;
}

static cc_status read_geometry_status(cc_ctx* ctx) {
  int counts[4] = {0, 0, 0, 0};
  int* dcounts = ctx->dim == 2 ? ctx->g2.counts : ctx->g3.counts;
  HIPCHK(ctx, hipMemcpyAsync(counts, dcounts, sizeof(counts), hipMemcpyDeviceToHost, ctx->stream),
         "geometry status copy");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "geometry build");
  if (counts[3] & 2) return fail(ctx, CC_EGEOM, "a cell is cut twice by the boundary");
  if (counts[3] & 1) return fail(ctx, CC_EGEOM, "master search cycles, leaves the domain or needs more than 4 hops");
  if (counts[3] & 4) return fail(ctx, CC_EGEOM, "a control volume has more members than supported");
  ctx->n_irr = counts[0];
  ctx->n_members = counts[1];
  ctx->n_solid = counts[2];
  return CC_OK;
}

cc_status bind_impl(cc_ctx* ctx, void* state0, void* state1, void* geom, void* scratch,
                    void* hip_stream) {
  if (!ctx) return CC_EINVAL;
  if (!state0 || !state1 || !geom || !scratch) return fail(ctx, CC_EINVAL, "null buffer");
  for (void* p : {state0, state1, geom, scratch})
    if ((uintptr_t)p % kAlign) return fail(ctx, CC_EINVAL, "buffers must be 256-byte aligned");
  ctx->state[0] = state0;
  ctx->state[1] = state1;
  ctx->cur = 0;
  ctx->geom = geom;
  ctx->scratch = scratch;
  ctx->stream = (hipStream_t)hip_stream;
  size_t b;
  if (ctx->dim == 2) layout_geo2d(ctx, (char*)geom, &b);
  else if (ctx->amr) layout_amr(ctx, (char*)geom, &b);
  else layout_geo3d(ctx, (char*)geom, &b);
  layout_scratch(ctx, (char*)scratch, &b);
  HIPCHK(ctx, hipMemsetAsync(scratch, 0, ctx->scratch_bytes, ctx->stream), "scratch clear");
  // solid cells are never written by a fixed-geometry step: both buffers
  // start at zero so that they read as empty on either side of the ping-pong
  HIPCHK(ctx, hipMemsetAsync(state0, 0, ctx->state_bytes, ctx->stream), "state clear");
  HIPCHK(ctx, hipMemsetAsync(state1, 0, ctx->state_bytes, ctx->stream), "state clear");
  HIPCHK(ctx, hipMemcpyAsync(ctx->s.body, ctx->body_state, 6 * sizeof(double),
                             hipMemcpyHostToDevice, ctx->stream), "body state upload");
  // a second stream for the cut control volumes, run beside the streaming
  // kernel (default priority, like the caller's stream)
  if (!ctx->side) {
    HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking), "side stream");
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming), "event");
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming), "event");
  }
  if (ctx->amr) {
    const AmrHost& H = *ctx->amrh;
    AmrDev& G = ctx->a3;
    hipError_t e = upload_amr_mesh(ctx);
    if (e == hipSuccess) e = launch_amr_tables(ctx);
    if (e != hipSuccess) return hip_fail(ctx, e, "octree upload");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "octree upload");
    // the generic 3D moment and mass kernels see the leaves through g3
    ctx->g3 = Geo3D{};
    ctx->g3.ncell = H.nleaf; ctx->g3.N = ctx->N; ctx->g3.nvel = ctx->nvel;
    ctx->g3.type = G.type; ctx->g3.master = G.master; ctx->g3.vcv = G.vcv;
    ctx->n_irr = H.n_irr; ctx->n_members = H.n_members; ctx->n_solid = H.n_solid;
    cc_status cst = check_cfl(ctx, true);
    if (cst != CC_OK) return cst;
    ctx->nstep = 0;
    ctx->bound = true;
    ctx->merged = false;
    ctx->mom_valid = false;
    return CC_OK;
  }
  hipError_t e = ctx->dim == 2 ? build_geometry_2d(ctx, ctx->g2, ctx->s.body) : build_geometry_3d(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "geometry kernels");
  if (ctx->dim == 2 && is_moving(ctx)) {
    e = build_geometry_2d(ctx, ctx->g2n, ctx->s.body);
    if (e != hipSuccess) return hip_fail(ctx, e, "geometry kernels");
    e = launch_moving_init_2d(ctx);
    if (e != hipSuccess) return hip_fail(ctx, e, "moving init");
  }
  cc_status st = read_geometry_status(ctx);
  if (st != CC_OK) return st;
  ctx->bound_geometry = true;
  st = check_cfl(ctx, true);
  if (st != CC_OK) return st;
  ctx->nstep = 0;
  ctx->bound = true;
  ctx->merged = false;
  ctx->mom_valid = false;
  return CC_OK;
}

// ---------------------------------------------------------------------------
// Binding without a caller scratch buffer.  The per-context records that
// cc_bind carves out of the caller's scratch buffer (moments of the current
// state, force and mass partials, rigid-body state, moving-body lists) live
// instead in a file-scope device array of fixed size, one copy per GPU.  Its
// device address is looked up once per device with hipGetSymbolAddress and
// only that address is handed to kernels and copies (the array's name is a
// host-side stand-in in host code).  The array holds the records of one
// bound context per GPU: binding another context to it takes it over, and
// the previous owner then reports CC_ESTATE until it is bound again.
namespace noalloc {
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex mu;
void* dev_ptr[kMaxDevices] = {};
cc_ctx* owner[kMaxDevices] = {};
}  // namespace noalloc

static void release_static_scratch(cc_ctx* ctx) {
  if (ctx->static_dev < 0) return;
  std::lock_guard<std::mutex> lock(noalloc::mu);
  if (noalloc::owner[ctx->static_dev] == ctx) noalloc::owner[ctx->static_dev] = nullptr;
  ctx->static_dev = -1;
}

cc_status bind_noalloc_impl(cc_ctx* ctx, void* state0, void* state1, void* geom, void* hip_stream) {
  if (!ctx) return CC_EINVAL;
  if (ctx->scratch_bytes > noalloc::kScratchBytes)
    return fail(ctx, CC_EINVAL, "this set-up needs " + std::to_string(ctx->scratch_bytes) +
                                    " scratch bytes; the static array holds " +
                                    std::to_string(noalloc::kScratchBytes));
  int dev = -1;
  HIPCHK(ctx, hipGetDevice(&dev), "current device");
  if (dev < 0 || dev >= noalloc::kMaxDevices) return fail(ctx, CC_EINVAL, "device index out of range");
  std::unique_lock<std::mutex> lock(noalloc::mu);
  if (!noalloc::dev_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc::scratch)), "static scratch address");
    if (!p) return fail(ctx, CC_EHIP, "static scratch address is null");
    noalloc::dev_ptr[dev] = p;
  }
  cc_ctx* prev = noalloc::owner[dev];
  if (prev && prev != ctx && prev->bound) {
    // hand over: finish the previous owner's work and keep its body state
    HIPCHK(ctx, hipStreamSynchronize(prev->stream), "previous owner's stream");
    if (!prev->amr_turning)
      HIPCHK(ctx, hipMemcpy(prev->body_state, prev->s.body, 6 * sizeof(double), hipMemcpyDeviceToHost),
             "previous owner's body state");
    prev->bound = false;
    prev->scratch_taken = true;
    prev->static_dev = -1;
  }
  noalloc::owner[dev] = ctx;
  void* ptr = noalloc::dev_ptr[dev];
  lock.unlock();
  ctx->static_dev = dev;
  ctx->scratch_taken = false;
  return bind_impl(ctx, state0, state1, geom, ptr, hip_stream);
}

// make the current state ready for a step: moments valid, control volumes merged
static cc_status prepare(cc_ctx* ctx) {
  if (ctx->amr) {
    // after a remap only the control volumes with several members (all
    // among the last group) need the merge and new records
    const int from = ctx->amr_leaf_records ? ctx->a3.nreg : 0;
    if (!ctx->merged) {
      HIPCHK(ctx, launch_amr_merge(ctx, from), "merge");
      ctx->merged = true;
      ctx->mom_valid = false;
    }
    if (!ctx->mom_valid) {
      HIPCHK(ctx, launch_amr_moments(ctx, from), "moments");
      ctx->mom_valid = true;
    }
    ctx->amr_leaf_records = false;
    return CC_OK;
  }
  if (ctx->dim == 3) {
    // 3D moment sums are taken of the merged control-volume values
    if (!ctx->merged) {
      HIPCHK(ctx, launch_merge_3d(ctx), "merge");
      ctx->merged = true;
      ctx->mom_valid = false;
    }
    if (!ctx->mom_valid) {
      HIPCHK(ctx, launch_moments_all_3d(ctx), "moments");
      ctx->mom_valid = true;
    }
    return CC_OK;
  }
  if (!ctx->mom_valid) {
    HIPCHK(ctx, launch_moments_all_2d(ctx), "moments");
    ctx->mom_valid = true;
  }
  if (!ctx->merged) {
    HIPCHK(ctx, launch_merge_2d(ctx), "merge");
    ctx->merged = true;
  }
  return CC_OK;
}

cc_status init_maxwellian_impl(cc_ctx* ctx) {
  if (!ctx) return CC_EINVAL;
  if (!ctx->bound) return not_bound(ctx);
  HIPCHK(ctx, ctx->amr ? launch_amr_init(ctx, nullptr)
                       : (ctx->dim == 2 ? launch_init_maxwellian_2d(ctx) : launch_init_maxwellian_3d(ctx)), "init");
  ctx->mom_valid = false;
  ctx->merged = false;
  ctx->amr_leaf_records = false;
  return prepare(ctx);
}

cc_status load_state_impl(cc_ctx* ctx, const double* f, const double* g) {
  if (!ctx || !f) return CC_EINVAL;
  if (!ctx->bound) return not_bound(ctx);
  if (ctx->dim == 2 && !g) return fail(ctx, CC_EINVAL, "g is required in 2D");
  HIPCHK(ctx, ctx->amr ? launch_amr_init(ctx, f)
                       : (ctx->dim == 2 ? launch_load_state_2d(ctx, f, g) : launch_load_state_3d(ctx, f)), "load");
  ctx->mom_valid = false;
  ctx->merged = false;
  ctx->amr_leaf_records = false;
  return prepare(ctx);
}

cc_status store_state_impl(const cc_ctx* ctx, double* f, double* g) {
  if (!ctx || !f) return CC_EINVAL;
  if (!ctx->bound) return CC_ESTATE;
  hipError_t e = ctx->dim == 2 ? launch_store_state_2d(ctx, f, g) : launch_store_state_3d(ctx, f);
  return e == hipSuccess ? CC_OK : CC_EHIP;
}

// One step of a body turning on the octree (Section 5, steps 1-7, then the
// mesh adapted to the body).  The host plans the step on the mesh of t^n
// (geometry at t^{n+1}, receiving control volumes), the kernels step the
// state, the torque sets the angular velocity of t^{n+1} (one
// synchronisation per step), the host builds the mesh of t^{n+1} and the
// remap kernel carries the state over.  row (device, nullable) = Fx, Fy,
// torque about the axis, mass of the state entering the step.
static cc_status amr_turning_step(cc_ctx* ctx, double* row) {
  AmrHost& H = *ctx->amrh;
  const double th = ctx->body_state[2], om = ctx->body_state[5];
  const double th1 = th + ctx->dt * om;
  std::string err;
  auto t0 = std::chrono::steady_clock::now();
  if (!plan_amr_move(ctx->cfg, ctx->body, th1, H, err)) return fail(ctx, CC_EGEOM, err);
  HIPCHK(ctx, upload_amr_plan(ctx), "step plan upload");
  auto t1 = std::chrono::steady_clock::now();
  cc_status st = prepare(ctx);
  if (st != CC_OK) return st;
  double* drow = row ? row : ctx->s.red + 4 * 128 + 4;
  HIPCHK(ctx, launch_amr_step(ctx, drow), "step");
  // the mesh of t^{n+1} depends only on the angle of t^{n+1}: it is built
  // on the host while the device runs the step
  auto t2 = std::chrono::steady_clock::now();
  // the mesh of two steps ago is recycled (its vectors keep their capacity)
  // held until the context takes it over, so that every early return
  // (including an exception) frees it; the build's future is destroyed
  // first and waits for the build to end
  std::unique_ptr<AmrHost> hold(ctx->amr_spare ? ctx->amr_spare : new (std::nothrow) AmrHost());
  ctx->amr_spare = nullptr;
  AmrHost* N1 = hold.get();
  if (!N1) return fail(ctx, CC_ENOMEM, "host allocation");
  std::string err1;
  double build_ms = 0.0;
  auto built = std::async(std::launch::async, [&] {
    auto b0 = std::chrono::steady_clock::now();
    const bool ok = build_octree_3d(ctx->cfg, ctx->body, th1, *N1, err1, &H);
    build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - b0).count();
    return ok;
  });
  double tq = 0.0;
  hipError_t he = hipMemcpyAsync(&tq, drow + 2, sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
  const bool ok1 = built.get();
  if (he != hipSuccess) return hip_fail(ctx, he, "step");
  if (!ok1) return fail(ctx, CC_EGEOM, err1);
  // the state carried over to the mesh of t^{n+1}
  AmrRemap R;
  build_amr_remap(H, *N1, ctx->cfg.amr_depth, R);
  if (N1->nleaf > H.cap_leaf || N1->nface > H.cap_face || (long long)R.src.size() > 2LL * H.cap_leaf)
    return fail(ctx, CC_ENOMEM, "the adapted mesh outgrew the buffers sized at cc_create");
  N1->cap_leaf = H.cap_leaf; N1->cap_face = H.cap_face;
  AmrDev& G = ctx->a3;
  HIPCHK(ctx, hipMemcpyAsync(G.sptr, R.sptr.data(), R.sptr.size() * sizeof(int), hipMemcpyHostToDevice, ctx->stream),
         "remap upload");
  if (!R.src.empty()) {
    HIPCHK(ctx, hipMemcpyAsync(G.src, R.src.data(), R.src.size() * sizeof(int), hipMemcpyHostToDevice, ctx->stream),
           "remap upload");
    HIPCHK(ctx, hipMemcpyAsync(G.wgt, R.wgt.data(), R.wgt.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream),
           "remap upload");
  }
  auto t3 = std::chrono::steady_clock::now();
  if (ctx->prof.on) {
    ctx->prof.host_ms[0] += std::chrono::duration<double, std::milli>(t1 - t0).count();
    ctx->prof.host_ms[1] += std::chrono::duration<double, std::milli>(t3 - t2).count();
    ctx->prof.host_ms[2] += build_ms;
    for (int k = 0; k < 3; ++k) ctx->prof.host_count[k] += 1;
  }
  // explicit Euler for the body: angle with the old angular velocity, the
  // angular velocity with the torque of t^n (free rotation)
  ctx->body_state[2] = th1;
  if (ctx->body.motion == CC_MOTION_FREE_ROTATION) ctx->body_state[5] = om + ctx->dt * tq / ctx->body.inertia;
  AmrHost* old = ctx->amrh;
  ctx->amrh = hold.release();
  ctx->ncell = N1->nleaf;
  // copies from pageable host memory return once the data is staged, so
  // the host vectors may change afterwards; the next step's planning on
  // the host then overlaps the remap on the device
  hipError_t e = upload_amr_mesh(ctx);
  if (e == hipSuccess) e = launch_amr_remap(ctx, (const double*)ctx->state[ctx->cur], (double*)ctx->state[1 - ctx->cur]);
  ctx->amr_spare = old;
  if (e != hipSuccess) return hip_fail(ctx, e, "mesh adaptation");
  ctx->cur = 1 - ctx->cur;
  ctx->n_irr = N1->n_irr; ctx->n_members = N1->n_members; ctx->n_solid = N1->n_solid;
  ctx->merged = false;
  ctx->mom_valid = false;
  ctx->amr_leaf_records = true;
  return CC_OK;
}

cc_status step_impl(cc_ctx* ctx, int nsteps, double* diag) {
  if (!ctx || nsteps < 0) return CC_EINVAL;
  if (!ctx->bound) return not_bound(ctx);
  cc_status st = prepare(ctx);
  if (st != CC_OK) return st;
  if (nsteps == 0) return CC_OK;
  bool moving = ctx->body.motion != CC_MOTION_FIXED && ctx->body.kind != CC_BODY_NONE;
  if (ctx->amr_turning) {
    for (int n = 0; n < nsteps; ++n) {
      st = amr_turning_step(ctx, diag ? diag + 4 * (size_t)n : nullptr);
      if (st != CC_OK) return st;
    }
    return CC_OK;
  }
  if (ctx->amr) {
    for (int n = 0; n < nsteps; ++n) {
      hipError_t e = launch_amr_step(ctx, diag ? diag + 4 * (size_t)n : nullptr);
      if (e != hipSuccess) return hip_fail(ctx, e, "step");
    }
    return CC_OK;
  }
  if (ctx->dim == 3) {
    // every step reduces its own force and mass rows
    for (int n = 0; n < nsteps; ++n) {
      hipError_t e = launch_step_3d(ctx, diag ? diag + 4 * (size_t)n : nullptr, nullptr);
      if (e != hipSuccess) return hip_fail(ctx, e, "step");
    }
    return CC_OK;
  }
  if (ctx->cfg.scheme == CC_SCHEME_IMEX && imex_fused_2d(ctx)) {
    // fused semi-implicit step; the force/mass partials of step n are
    // reduced by step n+1, as in the explicit step
    if (diag) HIPCHK(ctx, launch_mass_2d(ctx, diag + 3), "mass");
    for (int n = 0; n < nsteps; ++n) {
      bool red = diag && n > 0;
      hipError_t e = launch_imex_fused_2d(ctx, red, red ? diag + 4 * (size_t)(n - 1) : nullptr,
                                          red ? diag + 4 * (size_t)n + 3 : nullptr);
      if (e != hipSuccess) return hip_fail(ctx, e, "step");
    }
    if (diag) HIPCHK(ctx, launch_step_2d_flush(ctx, diag + 4 * (size_t)(nsteps - 1), nullptr), "reduce");
    return CC_OK;
  }
  if (ctx->cfg.scheme == CC_SCHEME_IMEX) {
    for (int n = 0; n < nsteps; ++n) {
      hipError_t e = launch_imex_step_2d(ctx, diag ? diag + 4 * (size_t)n : nullptr);
      if (e != hipSuccess) return hip_fail(ctx, e, "step");
    }
    return CC_OK;
  }
  if (diag) HIPCHK(ctx, launch_mass_2d(ctx, diag + 3), "mass");
  if (!moving) {
    // fused step; the force/mass partials of step n are reduced by step n+1
    for (int n = 0; n < nsteps; ++n) {
      bool red = diag && n > 0;
      hipError_t e = launch_step_2d_fused(ctx, red, red ? diag + 4 * (size_t)(n - 1) : nullptr,
                                          red ? diag + 4 * (size_t)n + 3 : nullptr, diag != nullptr);
      if (e != hipSuccess) return hip_fail(ctx, e, "step");
    }
    if (diag) HIPCHK(ctx, launch_step_2d_flush(ctx, diag + 4 * (size_t)(nsteps - 1), nullptr), "reduce");
    return CC_OK;
  }
  if (nsteps > 0) HIPCHK(ctx, launch_moving_prologue_2d(ctx), "moving geometry");
  for (int n = 0; n < nsteps; ++n) {
    double* frow = diag ? diag + 4 * (size_t)n : nullptr;
    double* mrow = (diag && n + 1 < nsteps) ? diag + 4 * (size_t)(n + 1) + 3 : nullptr;
    hipError_t e = launch_moving_step_2d(ctx, frow, mrow, n + 1 < nsteps);
    if (e != hipSuccess) return hip_fail(ctx, e, "step");
  }
  if (moving) {
    // a moving body rebuilds its geometry every step: report a rejected
    // geometry (one synchronisation per call)
    int bits[3] = {0, 0, 0};
    HIPCHK(ctx, hipMemcpyAsync(&bits[0], ctx->g2.counts + 3, sizeof(int), hipMemcpyDeviceToHost, ctx->stream), "status");
    HIPCHK(ctx, hipMemcpyAsync(&bits[1], ctx->g2n.counts + 3, sizeof(int), hipMemcpyDeviceToHost, ctx->stream), "status");
    HIPCHK(ctx, hipMemcpyAsync(&bits[2], ctx->s.gcount + 1, sizeof(int), hipMemcpyDeviceToHost, ctx->stream), "status");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "step sync");
    if (bits[0] | bits[1]) return fail(ctx, CC_EGEOM, "moving geometry rejected (cut twice, master search, members)");
    if (bits[2]) return fail(ctx, CC_EGEOM, "a cell appearing at the new time found no control volume");
  }
  return CC_OK;
}

cc_status set_tile_rows_impl(cc_ctx* ctx, int rows) {
  if (!ctx || rows < 0) return CC_EINVAL;
  ctx->seglen = rows;
  return CC_OK;
}

cc_status moments_impl(cc_ctx* ctx, double* out) {
  if (!ctx || !out) return CC_EINVAL;
  if (!ctx->bound) return not_bound(ctx);
  HIPCHK(ctx, ctx->dim == 2 ? launch_moments_out_2d(ctx, out) : launch_moments_out_3d(ctx, out), "moments");
  return CC_OK;
}

cc_status body_force_impl(cc_ctx* ctx, double out[4]) {
  if (!ctx || !out) return CC_EINVAL;
  if (!ctx->bound) return not_bound(ctx);
  if (ctx->amr) return fail(ctx, CC_EINVAL, "on the octree mesh the force comes with the diag rows of cc_step");
  cc_status st = prepare(ctx);
  if (st != CC_OK) return st;
  double* dev = ctx->s.red + 4 * 128 + 4;
  HIPCHK(ctx, ctx->dim == 2 ? launch_force_only_2d(ctx, dev) : launch_force_only_3d(ctx, dev), "force");
  HIPCHK(ctx, hipMemcpyAsync(out, dev, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream), "force copy");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "force sync");
  return CC_OK;
}

cc_status body_state_impl(cc_ctx* ctx, double out[6]) {
  if (!ctx || !out) return CC_EINVAL;
  if (!ctx->bound || ctx->amr_turning) {   // a turning body is advanced on the host
    memcpy(out, ctx->body_state, 6 * sizeof(double));
    return CC_OK;
  }
  HIPCHK(ctx, hipMemcpyAsync(ctx->body_state, ctx->s.body, 6 * sizeof(double),
                             hipMemcpyDeviceToHost, ctx->stream), "body copy");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "body sync");
  memcpy(out, ctx->body_state, 6 * sizeof(double));
  return CC_OK;
}

cc_status rigid_update_impl(cc_ctx* ctx, const double force[3], double torque) {
  if (!ctx || !force) return CC_EINVAL;
  double s[6];
  cc_status st = cc_body_state(ctx, s);
  if (st != CC_OK) return st;
  // eq. (motionDD_vit): explicit Euler on the velocities
  if (ctx->body.motion == CC_MOTION_FREE_ROTATION) {
    s[5] += ctx->dt * torque / ctx->body.inertia;
  } else if (ctx->body.motion == CC_MOTION_FIXED) {
    return fail(ctx, CC_EINVAL, "fixed body");
  }
  memcpy(ctx->body_state, s, sizeof(s));
  if (ctx->bound) {
    HIPCHK(ctx, hipMemcpyAsync(ctx->s.body, ctx->body_state, 6 * sizeof(double),
                               hipMemcpyHostToDevice, ctx->stream), "body upload");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "body sync");
  }
  return CC_OK;
}

cc_status geometry_export_impl(cc_ctx* ctx, int* type, int* master, double* lxm, double* lxp,
                               double* lym, double* lyp, double* lw, double* nwx, double* nwy,
                               double* rwx, double* rwy, double* sbar, double* scv) {
  if (!ctx) return CC_EINVAL;
  if (!ctx->bound) return not_bound(ctx);
  if (ctx->dim != 2) return fail(ctx, CC_EINVAL, "2D only");
  const Geo2D& G = ctx->g2;
  size_t n = ctx->ncell;
  struct { void* dst; const void* src; size_t sz; } cp[] = {
      {type, G.type, 4}, {master, G.master, 4}, {lxm, G.lxm, 8}, {lxp, G.lxp, 8},
      {lym, G.lym, 8}, {lyp, G.lyp, 8}, {lw, G.lw, 8}, {nwx, G.nwx, 8}, {nwy, G.nwy, 8},
      {rwx, G.rwx, 8}, {rwy, G.rwy, 8}, {sbar, G.sbar, 8}, {scv, G.scv, 8}};
  for (auto& c : cp)
    if (c.dst) HIPCHK(ctx, hipMemcpyAsync(c.dst, c.src, n * c.sz, hipMemcpyDeviceToHost, ctx->stream), "export");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "export sync");
  return CC_OK;
}

cc_status geometry_export3d_impl(cc_ctx* ctx, int* type, int* master, double* sxm, double* sxp,
                                 double* sym, double* syp, double* szm, double* szp, double* aw,
                                 double* nwx, double* nwy, double* nwz, double* rwx, double* rwy,
                                 double* rwz, double* vbar, double* vcv) {
  if (!ctx) return CC_EINVAL;
  if (!ctx->bound) return not_bound(ctx);
  if (ctx->dim != 3 || ctx->amr) return fail(ctx, CC_EINVAL, "uniform 3D grids only (octree: cc_amr_export)");
  const Geo3D& G = ctx->g3;
  size_t n = ctx->ncell;
  struct { void* dst; const void* src; size_t sz; } cp[] = {
      {type, G.type, 4}, {master, G.master, 4}, {sxm, G.sxm, 8}, {sxp, G.sxp, 8},
      {sym, G.sym, 8}, {syp, G.syp, 8}, {szm, G.szm, 8}, {szp, G.szp, 8}, {aw, G.aw, 8},
      {nwx, G.nwx, 8}, {nwy, G.nwy, 8}, {nwz, G.nwz, 8}, {rwx, G.rwx, 8}, {rwy, G.rwy, 8},
      {rwz, G.rwz, 8}, {vbar, G.vbar, 8}, {vcv, G.vcv, 8}};
  for (auto& c : cp)
    if (c.dst) HIPCHK(ctx, hipMemcpyAsync(c.dst, c.src, n * c.sz, hipMemcpyDeviceToHost, ctx->stream), "export");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "export sync");
  return CC_OK;
}

cc_status amr_counts_impl(cc_ctx* ctx, int* nleaf, int* nface) {
  if (!ctx) return CC_EINVAL;
  if (!ctx->amr) return fail(ctx, CC_EINVAL, "not an octree mesh");
  if (nleaf) *nleaf = ctx->amrh->nleaf;
  if (nface) *nface = ctx->amrh->nface;
  return CC_OK;
}

cc_status amr_export_impl(cc_ctx* ctx, int* lvl, int* ijk, int* type, int* master, double* vbar, double* vcv,
                          double* aw, double* S6) {
  if (!ctx) return CC_EINVAL;
  if (!ctx->amr) return fail(ctx, CC_EINVAL, "not an octree mesh");
  const AmrHost& H = *ctx->amrh;
  const size_t n = H.nleaf;
  if (lvl) memcpy(lvl, H.lvl.data(), n * sizeof(int));
  if (ijk) memcpy(ijk, H.ijk.data(), 3 * n * sizeof(int));
  if (type) memcpy(type, H.type.data(), n * sizeof(int));
  if (master) memcpy(master, H.master.data(), n * sizeof(int));
  if (vbar) memcpy(vbar, H.vbar.data(), n * sizeof(double));
  if (vcv) memcpy(vcv, H.vcv.data(), n * sizeof(double));
  if (aw) memcpy(aw, H.aw.data(), n * sizeof(double));
  if (S6) memcpy(S6, H.S6.data(), 6 * n * sizeof(double));
  return CC_OK;
}

cc_status amr_faces_impl(cc_ctx* ctx, int* fptr, int* fnb, int* fdir, double* farea) {
  if (!ctx) return CC_EINVAL;
  if (!ctx->amr) return fail(ctx, CC_EINVAL, "not an octree mesh");
  const AmrHost& H = *ctx->amrh;
  if (fptr) memcpy(fptr, H.fptr.data(), H.fptr.size() * sizeof(int));
  if (fnb) memcpy(fnb, H.fnb.data(), H.fnb.size() * sizeof(int));
  if (fdir) memcpy(fdir, H.fdir.data(), H.fdir.size() * sizeof(int));
  if (farea) memcpy(farea, H.farea.data(), H.farea.size() * sizeof(double));
  return CC_OK;
}

cc_status geometry_counts_impl(cc_ctx* ctx, int* n_irregular, int* n_members, int* n_solid) {
  if (!ctx) return CC_EINVAL;
  if (!ctx->bound) return not_bound(ctx);
  if (n_irregular) *n_irregular = ctx->n_irr;
  if (n_members) *n_members = ctx->n_members;
  if (n_solid) *n_solid = ctx->n_solid;
  return CC_OK;
}

cc_status profile_enable_impl(cc_ctx* ctx, int on) {
  if (!ctx) return CC_EINVAL;
  Prof& P = ctx->prof;
  if (on && P.start[0].empty()) {
    for (int k = 0; k < kProfKernels; ++k) {
      P.start[k].resize(kProfCap);
      P.stop[k].resize(kProfCap);
      for (int e = 0; e < kProfCap; ++e) {
        HIPCHK(ctx, hipEventCreate(&P.start[k][e]), "event create");
        HIPCHK(ctx, hipEventCreate(&P.stop[k][e]), "event create");
      }
    }
  }
  P.on = on != 0;
  for (int k = 0; k < kProfKernels; ++k) P.count[k] = 0;
  for (int k = 0; k < 3; ++k) { P.host_ms[k] = 0.0; P.host_count[k] = 0; }
  return CC_OK;
}

cc_status profile_read_impl(cc_ctx* ctx, int kernel, double* total_ms, int* launches) {
  if (!ctx || kernel < 0 || kernel >= kProfKernels + 3) return CC_EINVAL;
  Prof& P = ctx->prof;
  if (kernel >= kProfKernels) {   // host time of a turning body's step
    const int k = kernel - kProfKernels;
    if (total_ms) *total_ms = P.host_ms[k];
    if (launches) *launches = P.host_count[k];
    return CC_OK;
  }
  double tot = 0.0;
  if (P.count[kernel] > 0) HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "profile sync");
  for (int e = 0; e < P.count[kernel]; ++e) {
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, P.start[kernel][e], P.stop[kernel][e]), "elapsed");
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = P.count[kernel];
  return CC_OK;
}

// ---------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------
static const double kGamma = 5.0 / 3.0;

cc_status adjoint_workspace_bytes_impl(const cc_ctx* ctx, int nsteps, int ckpt_every, size_t* bytes) {
  if (!ctx || !bytes || nsteps < 1 || ckpt_every < 1) return CC_EINVAL;
  if (ctx->dim != 2 || is_moving(ctx)) return CC_EINVAL;
  *bytes = adjoint_workspace_bytes(ctx, nsteps, ckpt_every);
  return CC_OK;
}

cc_status adjoint_impl(cc_ctx* ctx, int nsteps, int ckpt_every, int objective, void* pool, double out[4]) {
  if (!ctx || !out || !pool || nsteps < 1 || ckpt_every < 1 || (objective != 0 && objective != 1))
    return CC_EINVAL;
  if (!ctx->bound) return not_bound(ctx);
  if (ctx->dim != 2 || is_moving(ctx)) return fail(ctx, CC_EINVAL, "the adjoint covers 2D fixed bodies");
  if (ctx->cfg.maxwellian != CC_MAXW_DIRECT || ctx->cfg.scheme != CC_SCHEME_EXPLICIT ||
      ctx->cfg.model != CC_MODEL_BGK)
    return fail(ctx, CC_EINVAL, "the adjoint is written for the explicit BGK scheme with the direct equilibrium");
  if ((uintptr_t)pool % kAlign) return fail(ctx, CC_EINVAL, "pool must be 256-byte aligned");
  cc_status st = cc_init_maxwellian(ctx);
  if (st != CC_OK) return st;
  double r[5];
  hipError_t e = adjoint_run_2d(ctx, nsteps, ckpt_every, objective, (char*)pool, r);
  if (e != hipSuccess) return hip_fail(ctx, e, "adjoint");
  // Mach number along the inflow direction: u = Ma sqrt(gamma T) e
  const double ux = ctx->cfg.inflow[1], uy = ctx->cfg.inflow[2], un = sqrt(ux * ux + uy * uy);
  const double ex = un > 0.0 ? ux / un : 1.0, ey = un > 0.0 ? uy / un : 0.0;
  out[0] = r[0];
  out[1] = r[1];
  out[2] = r[2];
  out[3] = sqrt(kGamma * ctx->cfg.inflow[4]) * (ex * r[3] + ey * r[4]);
  return CC_OK;
}

// ---------------------------------------------------------------------
// batched instances
// ---------------------------------------------------------------------
static const int kBatchMinRows = 4;
static const int kBatchRows[] = {8, 16, 32, 64, 128};

static cc_status batch_fail(cc_batch* b, cc_status st, const std::string& msg) {
  if (b) b->err = msg;
  return st;
}

static cc_status batch_upload_and_capture(cc_batch* b) {
  std::vector<char> d0, d1;
  std::vector<int2> tiles, cuts;
  batch_fill(b, d0, d1, tiles, cuts);
  if (tiles.size() > b->tile_cap || cuts.size() > b->cut_cap)
    return batch_fail(b, CC_ENOMEM, "batch work lists exceed the workspace");
  b->ncut = (int)cuts.size();
  hipError_t e;
  if ((e = hipMemcpyAsync(b->d_desc0, d0.data(), d0.size(), hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(b->d_desc1, d1.data(), d1.size(), hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
      (tiles.size() && (e = hipMemcpyAsync(b->d_tiles, tiles.data(), tiles.size() * sizeof(int2),
                                           hipMemcpyHostToDevice, b->stream)) != hipSuccess) ||
      (cuts.size() && (e = hipMemcpyAsync(b->d_cuts, cuts.data(), cuts.size() * sizeof(int2),
                                          hipMemcpyHostToDevice, b->stream)) != hipSuccess) ||
      (e = hipStreamSynchronize(b->stream)) != hipSuccess)
    return batch_fail(b, CC_EHIP, std::string("batch upload: ") + hipGetErrorString(e));
  // one step per ping-pong parity, recorded on a private capture stream with
  // side streams for the independent kernels (all at the default priority)
  // the capture stream and the side streams are destroyed on every exit
  struct Streams {
    hipStream_t cap = nullptr, side[4] = {nullptr, nullptr, nullptr, nullptr};
    ~Streams() {
      if (cap) hipStreamDestroy(cap);
      for (hipStream_t s : side)
        if (s) hipStreamDestroy(s);
    }
  } ss;
  if ((e = hipStreamCreateWithFlags(&ss.cap, hipStreamNonBlocking)) != hipSuccess)
    return batch_fail(b, CC_EHIP, "capture stream");
  for (int k = 0; k < 4; ++k)
    if ((e = hipStreamCreateWithFlags(&ss.side[k], hipStreamNonBlocking)) != hipSuccess)
      return batch_fail(b, CC_EHIP, "capture stream");
  hipStream_t cap = ss.cap;
  hipStream_t user = b->stream;
  for (int par = 0; par < 2; ++par) {
    if (b->exec[par]) { hipGraphExecDestroy(b->exec[par]); b->exec[par] = nullptr; }
    if (b->graph[par]) { hipGraphDestroy(b->graph[par]); b->graph[par] = nullptr; }
    b->stream = cap;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t le = batch_launch_step(b, par, ss.side, 4);
      e = hipStreamEndCapture(cap, &b->graph[par]);
      if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec[par], b->graph[par], nullptr, nullptr, 0);
    b->stream = user;
    if (e != hipSuccess) return batch_fail(b, CC_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  }
  b->base_cur.resize(b->ctx.size());
  for (size_t i = 0; i < b->ctx.size(); ++i) b->base_cur[i] = b->ctx[i]->cur;
  b->steps = 0;
  return CC_OK;
}

cc_status batch_create_impl(cc_ctx* const* ctxs, int n, cc_batch** out) {
  if (!ctxs || n < 1 || !out) return CC_EINVAL;
  *out = nullptr;
  // held until it is handed out, so that an exception does not leak it
  std::unique_ptr<cc_batch> hold(new (std::nothrow) cc_batch());
  cc_batch* b = hold.get();
  if (!b) return CC_ENOMEM;
  for (int i = 0; i < n; ++i) {
    cc_ctx* c = ctxs[i];
    bool ok = c && c->bound && c->dim == 2 && !is_moving(c) && c->cfg.maxwellian == CC_MAXW_DIRECT &&
              c->cfg.scheme == CC_SCHEME_EXPLICIT && c->cfg.model == CC_MODEL_BGK &&
              batch_supported_nch(batch_group_nch(c));
    for (int k = 0; k < i && ok; ++k) ok = ctxs[k] != c;
    if (ok && i > 0) ok = c->stream == ctxs[0]->stream;
    if (!ok) {
      fprintf(stderr, "ccdvm: batch instance %d must be a distinct bound 2D fixed-body context "
                      "(explicit, direct equilibrium) on the stream of instance 0\n", i);
      return CC_EINVAL;
    }
    b->ctx.push_back(c);
    int g = batch_group_nch(c);
    bool seen = false;
    for (int x : b->group_nch) seen |= x == g;
    if (!seen) b->group_nch.push_back(g);
  }
  std::sort(b->group_nch.begin(), b->group_nch.end());
  b->group_rows.assign(b->group_nch.size(), 16);   // until cc_batch_autotune picks per group
  b->stream = ctxs[0]->stream;
  for (cc_ctx* c : b->ctx) {
    b->tile_cap += (size_t)((c->nx + 3) / 4) * ((c->ny + kBatchMinRows - 1) / kBatchMinRows);
    b->cut_cap += c->n_irr;
  }
  size_t desc = align_up(n * batch_desc_bytes());
  b->dev_bytes = 2 * desc + align_up(b->tile_cap * sizeof(int2)) + align_up((b->cut_cap + 1) * sizeof(int2));
  *out = hold.release();
  return CC_OK;
}

cc_status batch_workspace_bytes_impl(const cc_batch* b, size_t* bytes) {
  if (!b || !bytes) return CC_EINVAL;
  *bytes = b->dev_bytes;
  return CC_OK;
}

cc_status batch_bind_impl(cc_batch* b, void* workspace) {
  if (!b || !workspace) return CC_EINVAL;
  if ((uintptr_t)workspace % kAlign) return batch_fail(b, CC_EINVAL, "workspace must be 256-byte aligned");
  b->dev = (char*)workspace;
  size_t desc = align_up(b->ctx.size() * batch_desc_bytes());
  b->d_desc0 = b->dev;
  b->d_desc1 = b->dev + desc;
  b->d_tiles = (int2*)(b->dev + 2 * desc);
  b->d_cuts = (int2*)(b->dev + 2 * desc + align_up(b->tile_cap * sizeof(int2)));
  for (cc_ctx* c : b->ctx) {
    cc_status st = prepare(c);
    if (st != CC_OK) return batch_fail(b, st, "instance preparation failed: " + c->err);
  }
  cc_status st = batch_upload_and_capture(b);
  if (st != CC_OK) return st;
  b->bound = true;
  return CC_OK;
}

cc_status batch_autotune_impl(cc_batch* b, int trial_steps, int* rows_out) {
  if (!b || trial_steps < 1) return CC_EINVAL;
  if (!b->bound) return batch_fail(b, CC_ESTATE, "cc_batch_bind first");
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return batch_fail(b, CC_EHIP, "events");
  for (size_t g = 0; g < b->group_nch.size(); ++g) {
    double best = 1e300;
    int best_rows = 0;
    for (int rows : kBatchRows) {
      b->group_rows[g] = rows;
      cc_status st = batch_upload_and_capture(b);
      if (st != CC_OK) return st;
      batch_launch_group(b, (int)g);   // warm-up
      hipEventRecord(e0, b->stream);
      for (int k = 0; k < trial_steps; ++k) batch_launch_group(b, (int)g);
      hipEventRecord(e1, b->stream);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) { best = ms; best_rows = rows; }
    }
    b->group_rows[g] = best_rows;
    if (rows_out) rows_out[g] = best_rows;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  // the trials advanced the regular cells of the ping-pong targets only, but
  // rewrote the regular cells' stored moments: recompute those from the
  // current states (the cut and merged control volumes keep theirs)
  for (cc_ctx* c : b->ctx) {
    cc_status st = prepare(c);
    if (st != CC_OK) return batch_fail(b, st, "instance preparation failed");
    if (launch_moments_all_2d(c, true) != hipSuccess) return batch_fail(b, CC_EHIP, "moments");
  }
  return batch_upload_and_capture(b);
}

cc_status batch_groups_impl(const cc_batch* b, int* ngroups, int* chunks, int* rows) {
  if (!b || !ngroups) return CC_EINVAL;
  *ngroups = (int)b->group_nch.size();
  for (size_t g = 0; g < b->group_nch.size(); ++g) {
    if (chunks) chunks[g] = b->group_nch[g];
    if (rows) rows[g] = b->group_rows[g];
  }
  return CC_OK;
}

cc_status batch_step_impl(cc_batch* b, int nsteps) {
  if (!b || nsteps < 0) return CC_EINVAL;
  if (!b->bound) return batch_fail(b, CC_ESTATE, "cc_batch_bind first");
  bool stale = false;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    cc_ctx* c = b->ctx[i];
    stale |= c->cur != (b->base_cur[i] ^ (int)(b->steps & 1));
    cc_status st = prepare(c);
    if (st != CC_OK) return batch_fail(b, st, "instance preparation failed");
  }
  if (stale) {
    cc_status st = batch_upload_and_capture(b);
    if (st != CC_OK) return st;
  }
  for (int k = 0; k < nsteps; ++k) {
    hipError_t e = hipGraphLaunch(b->exec[(b->steps + k) & 1], b->stream);
    if (e != hipSuccess) return batch_fail(b, CC_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
  }
  b->steps += nsteps;
  for (cc_ctx* c : b->ctx) {
    c->cur ^= nsteps & 1;
    c->nstep += nsteps;
  }
  return CC_OK;
}

cc_status batch_adjoint_workspace_bytes_impl(const cc_batch* b, int nsteps, int K, size_t* bytes) {
  if (!b || !bytes || nsteps < 1 || K < 1) return CC_EINVAL;
  *bytes = batch_adjoint_workspace_bytes(b, nsteps, K);
  return CC_OK;
}

cc_status batch_adjoint_impl(cc_batch* b, int nsteps, int K, int objective, void* ws, double* out) {
  if (!b || !ws || !out || nsteps < 1 || K < 1 || (objective != 0 && objective != 1)) return CC_EINVAL;
  if (!b->bound) return batch_fail(b, CC_ESTATE, "cc_batch_bind first");
  if ((uintptr_t)ws % kAlign) return batch_fail(b, CC_EINVAL, "workspace must be 256-byte aligned");
  for (cc_ctx* c : b->ctx) {
    if (!c->bound) return batch_fail(b, CC_ESTATE, "an instance is no longer bound");
    if (c->cfg.model != CC_MODEL_BGK)
      return batch_fail(b, CC_EINVAL, "the adjoint is written for the BGK model");
    cc_status st = cc_init_maxwellian(c);
    if (st != CC_OK) return batch_fail(b, st, "instance initialisation failed: " + c->err);
  }
  std::vector<double> r(5 * b->ctx.size());
  hipError_t e = batch_adjoint_run_2d(b, nsteps, K, objective, (char*)ws, r.data());
  if (e != hipSuccess) return batch_fail(b, CC_EHIP, std::string("batched adjoint: ") + hipGetErrorString(e));
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    const cc_ctx* c = b->ctx[i];
    // Mach number along the inflow direction, as cc_adjoint
    const double ux = c->cfg.inflow[1], uy = c->cfg.inflow[2], un = sqrt(ux * ux + uy * uy);
    const double ex = un > 0.0 ? ux / un : 1.0, ey = un > 0.0 ? uy / un : 0.0;
    out[4 * i + 0] = r[5 * i + 0];
    out[4 * i + 1] = r[5 * i + 1];
    out[4 * i + 2] = r[5 * i + 2];
    out[4 * i + 3] = sqrt(kGamma * c->cfg.inflow[4]) * (ex * r[5 * i + 3] + ey * r[5 * i + 4]);
  }
  return CC_OK;
}

}  // namespace

extern "C" {

cc_status cc_create(const cc_config* cfg, const cc_body* body, cc_ctx** out) {
  return no_throw(nullptr, [&] { return create_impl(cfg, body, out); });
}

cc_status cc_workspace_bytes(const cc_ctx* ctx, size_t* state_bytes, size_t* geom_bytes,
                             size_t* scratch_bytes) {
  return no_throw(nullptr, [&] { return workspace_bytes_impl(ctx, state_bytes, geom_bytes, scratch_bytes); });
}

cc_status cc_dt(const cc_ctx* ctx, double* dt) {
  return no_throw(nullptr, [&] { return dt_impl(ctx, dt); });
}

cc_status cc_bind(cc_ctx* ctx, void* state0, void* state1, void* geom, void* scratch, void* hip_stream) {
  return no_throw(ctx ? &ctx->err : nullptr, [&] {
    if (ctx) {
      release_static_scratch(ctx);
      ctx->scratch_taken = false;
    }
    return bind_impl(ctx, state0, state1, geom, scratch, hip_stream);
  });
}

cc_status cc_bind_noalloc(cc_ctx* ctx, void* state0, void* state1, void* geom, void* hip_stream) {
  return no_throw(ctx ? &ctx->err : nullptr,
                  [&] { return bind_noalloc_impl(ctx, state0, state1, geom, hip_stream); });
}

cc_status cc_cfl_number(const cc_ctx* ctx, double out[3]) {
  return no_throw(nullptr, [&] { return cfl_number_impl(ctx, out); });
}

cc_status cc_init_maxwellian(cc_ctx* ctx) {
  return no_throw(ctx ? &ctx->err : nullptr, [&] { return init_maxwellian_impl(ctx); });
}

cc_status cc_load_state(cc_ctx* ctx, const double* f, const double* g) {
  return no_throw(ctx ? &ctx->err : nullptr, [&] { return load_state_impl(ctx, f, g); });
}

cc_status cc_store_state(const cc_ctx* ctx, double* f, double* g) {
  return no_throw(nullptr, [&] { return store_state_impl(ctx, f, g); });
}

cc_status cc_step(cc_ctx* ctx, int nsteps, double* diag) {
  return no_throw(ctx ? &ctx->err : nullptr, [&] { return step_impl(ctx, nsteps, diag); });
}

cc_status cc_set_tile_rows(cc_ctx* ctx, int rows) {
  return no_throw(ctx ? &ctx->err : nullptr, [&] { return set_tile_rows_impl(ctx, rows); });
}

cc_status cc_moments(cc_ctx* ctx, double* out) {
  return no_throw(ctx ? &ctx->err : nullptr, [&] { return moments_impl(ctx, out); });
}

cc_status cc_body_force(cc_ctx* ctx, double out[4]) {
  return no_throw(ctx ? &ctx->err : nullptr, [&] { return body_force_impl(ctx, out); });
}

cc_status cc_body_state(cc_ctx* ctx, double out[6]) {
  return no_throw(ctx ? &ctx->err : nullptr, [&] { return body_state_impl(ctx, out); });
}

cc_status cc_rigid_update(cc_ctx* ctx, const double force[3], double torque) {
  return no_throw(ctx ? &ctx->err : nullptr, [&] { return rigid_update_impl(ctx, force, torque); });
}

cc_status cc_geometry_export(cc_ctx* ctx, int* type, int* master, double* lxm, double* lxp, double* lym,
                             double* lyp, double* lw, double* nwx, double* nwy, double* rwx, double* rwy,
                             double* sbar, double* scv) {
  return no_throw(ctx ? &ctx->err : nullptr,
                  [&] { return geometry_export_impl(ctx, type, master, lxm, lxp, lym, lyp, lw, nwx, nwy, rwx,
                                                    rwy, sbar, scv); });
}

cc_status cc_geometry_export3d(cc_ctx* ctx, int* type, int* master, double* sxm, double* sxp, double* sym,
                               double* syp, double* szm, double* szp, double* aw, double* nwx, double* nwy,
                               double* nwz, double* rwx, double* rwy, double* rwz, double* vbar,
                               double* vcv) {
  return no_throw(ctx ? &ctx->err : nullptr, [&] {
    return geometry_export3d_impl(ctx, type, master, sxm, sxp, sym, syp, szm, szp, aw, nwx, nwy, nwz, rwx,
                                  rwy, rwz, vbar, vcv);
  });
}

cc_status cc_amr_counts(cc_ctx* ctx, int* nleaf, int* nface) {
  return no_throw(ctx ? &ctx->err : nullptr, [&] { return amr_counts_impl(ctx, nleaf, nface); });
}

cc_status cc_amr_export(cc_ctx* ctx, int* lvl, int* ijk, int* type, int* master, double* vbar, double* vcv,
                        double* aw, double* S6) {
  return no_throw(ctx ? &ctx->err : nullptr,
                  [&] { return amr_export_impl(ctx, lvl, ijk, type, master, vbar, vcv, aw, S6); });
}

cc_status cc_amr_faces(cc_ctx* ctx, int* fptr, int* fnb, int* fdir, double* farea) {
  return no_throw(ctx ? &ctx->err : nullptr, [&] { return amr_faces_impl(ctx, fptr, fnb, fdir, farea); });
}

cc_status cc_geometry_counts(cc_ctx* ctx, int* n_irregular, int* n_members, int* n_solid) {
  return no_throw(ctx ? &ctx->err : nullptr,
                  [&] { return geometry_counts_impl(ctx, n_irregular, n_members, n_solid); });
}

cc_status cc_profile_enable(cc_ctx* ctx, int on) {
  return no_throw(ctx ? &ctx->err : nullptr, [&] { return profile_enable_impl(ctx, on); });
}

cc_status cc_profile_read(cc_ctx* ctx, int kernel, double* total_ms, int* launches) {
  return no_throw(ctx ? &ctx->err : nullptr,
                  [&] { return profile_read_impl(ctx, kernel, total_ms, launches); });
}

cc_status cc_adjoint_workspace_bytes(const cc_ctx* ctx, int nsteps, int ckpt_every, size_t* bytes) {
  return no_throw(nullptr, [&] { return adjoint_workspace_bytes_impl(ctx, nsteps, ckpt_every, bytes); });
}

cc_status cc_adjoint(cc_ctx* ctx, int nsteps, int ckpt_every, int objective, void* pool, double out[4]) {
  return no_throw(ctx ? &ctx->err : nullptr,
                  [&] { return adjoint_impl(ctx, nsteps, ckpt_every, objective, pool, out); });
}

cc_status cc_batch_create(cc_ctx* const* ctxs, int n, cc_batch** out) {
  return no_throw(nullptr, [&] { return batch_create_impl(ctxs, n, out); });
}

cc_status cc_batch_workspace_bytes(const cc_batch* b, size_t* bytes) {
  return no_throw(nullptr, [&] { return batch_workspace_bytes_impl(b, bytes); });
}

cc_status cc_batch_bind(cc_batch* b, void* workspace) {
  return no_throw(b ? &b->err : nullptr, [&] { return batch_bind_impl(b, workspace); });
}

cc_status cc_batch_autotune(cc_batch* b, int trial_steps, int* rows_out) {
  return no_throw(b ? &b->err : nullptr, [&] { return batch_autotune_impl(b, trial_steps, rows_out); });
}

cc_status cc_batch_groups(const cc_batch* b, int* ngroups, int* chunks, int* rows) {
  return no_throw(nullptr, [&] { return batch_groups_impl(b, ngroups, chunks, rows); });
}

cc_status cc_batch_step(cc_batch* b, int nsteps) {
  return no_throw(b ? &b->err : nullptr, [&] { return batch_step_impl(b, nsteps); });
}

void cc_destroy(cc_ctx* ctx) {
  if (!ctx) return;
  release_static_scratch(ctx);
  for (int k = 0; k < kProfKernels; ++k) {
    for (hipEvent_t e : ctx->prof.start[k]) hipEventDestroy(e);
    for (hipEvent_t e : ctx->prof.stop[k]) hipEventDestroy(e);
  }
  if (ctx->fork) hipEventDestroy(ctx->fork);
  if (ctx->join) hipEventDestroy(ctx->join);
  if (ctx->side) hipStreamDestroy(ctx->side);
  delete ctx->amrh;
  delete ctx->amr_spare;
  delete ctx;
}

const char* cc_last_error(const cc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

cc_status cc_batch_adjoint_workspace_bytes(const cc_batch* b, int nsteps, int ckpt_every, size_t* bytes) {
  return no_throw(nullptr, [&] { return batch_adjoint_workspace_bytes_impl(b, nsteps, ckpt_every, bytes); });
}

cc_status cc_batch_adjoint(cc_batch* b, int nsteps, int ckpt_every, int objective, void* workspace,
                           double* out) {
  return no_throw(b ? &b->err : nullptr,
                  [&] { return batch_adjoint_impl(b, nsteps, ckpt_every, objective, workspace, out); });
}

const char* cc_batch_last_error(const cc_batch* b) { return b ? b->err.c_str() : "null batch"; }

void cc_batch_destroy(cc_batch* b) {
  if (!b) return;
  for (int par = 0; par < 2; ++par) {
    if (b->exec[par]) hipGraphExecDestroy(b->exec[par]);
    if (b->graph[par]) hipGraphDestroy(b->graph[par]);
  }
  delete b;
}

}  // extern "C"
