// Octree mesh around a fixed body in 3D (Section 5.1, octree procedure) and
// its explicit step.
//
// Mesh (built once, on the host, when the context is created): the coarse
// grid cfg.n is refined near the boundary; a cell of depth d is divided in 8
// when the distance from its centre to the boundary (|level set|) is below
// band * dx / 2^d, dx the largest coarse spacing, and d < amr_depth, so the
// finest depth is amr_depth.  Leaves are stored in Z-order of their lower
// corner (finest-level units), which keeps face neighbours close in memory.
// Each leaf lists its faces in the order x-, x+, y-, y+, z-, z+: the leaf
// across (same depth, one coarser, or the four of the next finer depth) or
// the farfield, with the face's gas area (across a change of depth, the
// finer leaf's face).  Cut cells lie at the finest depth, where the leaves
// carry the uniform grid's cut-cell geometry (cellgeom3d.h) and master
// search; depth jumps of more than one, cut cells above the finest depth or
// a master search across a change of depth reject the mesh.
//
// Step (eq. eq-schema3D on the leaves): one wave per control volume reads
// its value (members hold it), gathers the upwind fluxes of its members'
// face lists and wall faces, relaxes toward the separable Maxwellian of the
// moments it stored the step before, writes the new value to every member
// and sums the moments of that value for the next step.  Velocities are
// walked in passes of RC per lane so that one face's loads of a pass are
// independent (memory-level parallelism on the gather).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <string>
#include <vector>

#include "ccdvm_impl.h"

#pragma clang fp contract(off)

#include "cellgeom3d.h"
#include "hostpool.h"

namespace ccdvm {

// ---------------------------------------------------------------------
// host builder
// ---------------------------------------------------------------------
namespace {

// bit b of x (b < 21) to bit 3b
uint64_t spread_bits3(uint64_t x) {
  x &= 0x1fffffULL;
  x = (x | x << 32) & 0x1f00000000ffffULL;
  x = (x | x << 16) & 0x1f0000ff0000ffULL;
  x = (x | x << 8) & 0x100f00f00f00f00fULL;
  x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
  x = (x | x << 2) & 0x1249249249249249ULL;
  return x;
}

uint64_t morton3(uint64_t i, uint64_t j, uint64_t k) {
  return spread_bits3(i) | (spread_bits3(j) << 1) | (spread_bits3(k) << 2);
}

// the leaf containing the lower corner of the depth-l cell (i, j, k), or -1
// outside the domain (from the finest-level map)
int leaf_at(const AmrHost& H, int D, int l, int i, int j, int k) {
  if (l < 0 || i < 0 || j < 0 || k < 0) return -1;
  const int sh = D - l;
  const long long I = (long long)i << sh, J = (long long)j << sh, K = (long long)k << sh;
  if (I >= H.nf[0] || J >= H.nf[1] || K >= H.nf[2]) return -1;
  return H.fine[(size_t)((K * H.nf[1] + J) * H.nf[0] + I)];
}

// the leaf of depth l at (i, j, k), or -1
int find_leaf(const AmrHost& H, int D, int l, int i, int j, int k) {
  const int y = leaf_at(H, D, l, i, j, k);
  return y >= 0 && H.lvl[y] == l ? y : -1;
}

BodyDev body_at(const cc_body& body, double theta) {
  BodyDev B{};
  B.kind = body.kind;
  B.cx = body.center[0]; B.cy = body.center[1]; B.cz = body.center[2];
  B.a = body.axes[0]; B.b = body.axes[1]; B.c = body.axes[2];
  B.theta = theta;
  B.ct = cos(theta); B.st = sin(theta);
  B.t_wall = body.t_wall;
  return B;
}

// Geometry of a cell of depth l far from the boundary (all 8 vertices on
// one side): the per-cell construction gives the same tables whatever the
// vertex values, so it is computed once per depth and side.
struct FarCells {
  CellGeo3 g[9][2];
  FarCells(const AmrHost& H, int D) {
    for (int l = 0; l <= D; ++l)
      for (int gas = 0; gas < 2; ++gas) {
        double h[3], qv[8];
        for (int d = 0; d < 3; ++d) h[d] = H.hf[d] * (double)(1 << (D - l));
        for (int t = 0; t < 8; ++t) qv[t] = gas ? 1.0 : -1.0;
        cell_geometry_3d(qv, h, 1e-12 * H.hf[0], g[l][gas]);
      }
  }
  const CellGeo3& get(int l, bool gas) const { return g[l][gas]; }
};

// geometry of leaf q with the body B: its 8 vertex values (clamped as on
// the uniform grid) and the uniform grid's per-cell construction at the
// leaf's size; A0 = lower corner in finest units.  The level sets are
// signed distances (1-Lipschitz): a leaf whose centre is farther from the
// boundary than its half-diagonal (with a margin far above rounding) has
// all vertices on the centre's side and takes the far-cell tables.
void leaf_geometry(const cc_config& cfg, const AmrHost& H, const BodyDev& B, int q, CellGeo3& g, int A0[3],
                   const FarCells& far) {
  const int sh = cfg.amr_depth - H.lvl[q];
  for (int d = 0; d < 3; ++d) A0[d] = H.ijk[3 * (size_t)q + d] << sh;
  double qv[8], h[3];
  for (int d = 0; d < 3; ++d) h[d] = H.hf[d] * (double)(1 << sh);
  const double pc = level_set_3d(B, cfg.lo[0] + (A0[0] + 0.5 * (1 << sh)) * H.hf[0],
                                 cfg.lo[1] + (A0[1] + 0.5 * (1 << sh)) * H.hf[1],
                                 cfg.lo[2] + (A0[2] + 0.5 * (1 << sh)) * H.hf[2]);
  const double hd = 0.5 * sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
  if (fabs(pc) > hd * (1.0 + 1e-9) + 1e-12 * H.hf[0]) {
    g = far.get(H.lvl[q], pc > 0.0);
    return;
  }
  for (int t = 0; t < 8; ++t) {
    // corner t at ((t >> 2) & 1, (t >> 1) & 1, t & 1) in units of the leaf size
    const int a = A0[0] + (((t >> 2) & 1) << sh), b = A0[1] + (((t >> 1) & 1) << sh), c = A0[2] + ((t & 1) << sh);
    qv[t] = clamp_vertex(level_set_3d(B, cfg.lo[0] + a * H.hf[0], cfg.lo[1] + b * H.hf[1], cfg.lo[2] + c * H.hf[2]),
                         H.hf[0]);
  }
  cell_geometry_3d(qv, h, 1e-12 * H.hf[0], g);
}

// Control volumes in kernel order: first the regular ones (one member, no
// wall face; simple ones, with one face entry per direction in direction
// order, before the others), then the cut or merged ones, each group in
// leaf order; with a turning body the control volumes marked in `changed`
// (volume or receivers differ between t^n and t^{n+1}) join the last group.
bool order_cvs(AmrHost& H, const std::vector<char>* changed, std::string& err) {
  const int n = H.nleaf;
  HostPool& pool = HostPool::get();
  const int C = HostPool::kChunk;
  const int nchunk = (n + C - 1) / C;
  // members per master: the master itself (leaves in parallel), then the
  // other members ("foreign", few), gathered per chunk and added in leaf order
  std::vector<int> cnt(n);
  std::vector<std::vector<int>> foreign(nchunk);
  pool.run(n, [&](int b, int e) {
    std::vector<int>& f = foreign[b / C];
    for (int q = b; q < e; ++q) {
      const int m = H.master[q];
      cnt[q] = m == q ? 1 : 0;
      if (m >= 0 && m != q) f.push_back(q);
    }
  });
  std::vector<int> fq;
  for (const std::vector<int>& f : foreign) fq.insert(fq.end(), f.begin(), f.end());
  for (int q : fq) cnt[H.master[q]]++;
  auto kind_of = [&](int q) {
    if (cnt[q] != 1 || H.aw[q] > 0.0 || (changed && (*changed)[q])) return 2;
    if (H.fptr[q + 1] - H.fptr[q] != 6) return 1;
    for (int t = 0; t < 6; ++t) if (H.fdir[H.fptr[q] + t] != t) return 1;
    return 0;
  };
  // kind of every master (-1 for other leaves) and the count of each kind
  // per chunk, leaves in parallel
  std::vector<signed char> kind(n);
  std::vector<int> kc(3 * (size_t)nchunk, 0);
  std::atomic<bool> too_many{false};
  pool.run(n, [&](int b, int e) {
    int k3[3] = {0, 0, 0};
    for (int q = b; q < e; ++q) {
      const int kd = H.master[q] == q ? kind_of(q) : -1;
      kind[q] = (signed char)kd;
      if (kd >= 0) k3[kd]++;
      if (H.master[q] == q && cnt[q] > kMaxMembers) too_many = true;
    }
    for (int t = 0; t < 3; ++t) kc[3 * (size_t)(b / C) + t] = k3[t];
  });
  if (too_many) { err = "a control volume has more members than supported"; return false; }
  // control volumes in kind order, each kind in leaf order: chunk c's
  // masters of kind t start at the kinds before t plus chunks before c
  std::vector<int> start(3 * (size_t)nchunk);
  int at = 0;
  for (int t = 0; t < 3; ++t) {
    if (t == 1) H.nsimple = at;
    if (t == 2) H.nreg = at;
    for (int c = 0; c < nchunk; ++c) { start[3 * (size_t)c + t] = at; at += kc[3 * (size_t)c + t]; }
  }
  const int ncv = at;
  H.cv.resize(ncv);
  std::vector<int> slot(n);
  pool.run(n, [&](int b, int e) {
    int pos[3];
    for (int t = 0; t < 3; ++t) pos[t] = start[3 * (size_t)(b / C) + t];
    for (int q = b; q < e; ++q) {
      const int kd = kind[q];
      slot[q] = kd >= 0 ? pos[kd] : -1;
      if (kd >= 0) H.cv[pos[kd]++] = q;
    }
  });
  // member offsets: a prefix sum over the control volumes, chunks in parallel
  const int ncc = (ncv + C - 1) / C;
  std::vector<int> csum(ncc + 1, 0);
  pool.run(ncv, [&](int b, int e) {
    int sum = 0;
    for (int s = b; s < e; ++s) sum += cnt[H.cv[s]];
    csum[b / C + 1] = sum;
  });
  for (int c = 0; c < ncc; ++c) csum[c + 1] += csum[c];
  H.cvptr.resize(ncv + 1);
  H.cvptr[0] = 0;
  pool.run(ncv, [&](int b, int e) {
    int off = csum[b / C];
    for (int s = b; s < e; ++s) { off += cnt[H.cv[s]]; H.cvptr[s + 1] = off; }
  });
  // members in leaf order: a lone master is its only member; a master with
  // foreign members takes its place among them
  H.cvmem.resize(ncv ? H.cvptr[ncv] : 0);
  pool.run(ncv, [&](int b, int e) {
    for (int s = b; s < e; ++s) H.cvmem[H.cvptr[s]] = H.cv[s];
  });
  if (!fq.empty()) {
    std::vector<int> fill(ncv, 0), touched;
    std::vector<char> placed(ncv, 0);
    for (int q : fq) {   // ascending
      const int m = H.master[q], sl = slot[m];
      if (fill[sl] == 0 && !placed[sl]) touched.push_back(sl);
      if (!placed[sl] && m < q) { H.cvmem[H.cvptr[sl] + fill[sl]++] = m; placed[sl] = 1; }
      H.cvmem[H.cvptr[sl] + fill[sl]++] = q;
    }
    // a master above all its foreign members comes last
    for (int sl : touched)
      if (!placed[sl]) H.cvmem[H.cvptr[sl] + fill[sl]++] = H.cv[sl];
  }
  return true;
}

}  // namespace

bool build_octree_3d(const cc_config& cfg, const cc_body& body, double theta, AmrHost& H, std::string& err,
                     const AmrHost* prev) {
  const int D = cfg.amr_depth;
  const BodyDev B = body_at(body, theta);
  double h0[3];
  for (int d = 0; d < 3; ++d) {
    H.n0[d] = cfg.n[d];
    h0[d] = (cfg.hi[d] - cfg.lo[d]) / cfg.n[d];
    H.hf[d] = (cfg.hi[d] - cfg.lo[d]) / (double)(cfg.n[d] << D);
  }
  const double Dx = std::max(h0[0], std::max(h0[1], h0[2]));
  const double band = cfg.amr_band > 0.0 ? cfg.amr_band : 2.0 * sqrt(2.0);
  HostPool& pool = HostPool::get();
  // refinement of every coarse cell by the criterion, coarse cells in
  // parallel and in Z-order, each walked depth first with the children in
  // Z-order: the leaves come out in the Z-order of their lower corners
  struct C4 { int l, i, j, k; };
  const int n0 = cfg.n[0] * cfg.n[1] * cfg.n[2];
  AmrBuildScratch& X = H.scratch;
  std::vector<std::pair<uint64_t, int>>& corder = X.corder;
  if ((int)corder.size() != n0) {
    corder.resize(n0);
    for (int c0 = 0; c0 < n0; ++c0)
      corder[c0] = {morton3(c0 % cfg.n[0], (c0 / cfg.n[0]) % cfg.n[1], c0 / (cfg.n[0] * cfg.n[1])), c0};
    std::sort(corder.begin(), corder.end());
  }
  std::vector<std::vector<int>>& part = X.part;
  part.resize((n0 + HostPool::kChunk - 1) / HostPool::kChunk);
  pool.run(n0, [&](int b, int e) {
    std::vector<int>& out = part[b / HostPool::kChunk];
    out.clear();
    std::vector<C4> stack;
    for (int z0 = b; z0 < e; ++z0) {
      const int c0 = corder[z0].second;
      stack.push_back({0, c0 % cfg.n[0], (c0 / cfg.n[0]) % cfg.n[1], c0 / (cfg.n[0] * cfg.n[1])});
      while (!stack.empty()) {
        const C4 c = stack.back();
        stack.pop_back();
        const double s = 1.0 / (double)(1 << c.l);
        const double x = cfg.lo[0] + (c.i + 0.5) * h0[0] * s, y = cfg.lo[1] + (c.j + 0.5) * h0[1] * s,
                     z = cfg.lo[2] + (c.k + 0.5) * h0[2] * s;
        if (c.l < D && fabs(level_set_3d(B, x, y, z)) < band * Dx * s) {
          for (int t = 7; t >= 0; --t)
            stack.push_back({c.l + 1, 2 * c.i + (t & 1), 2 * c.j + ((t >> 1) & 1), 2 * c.k + ((t >> 2) & 1)});
        } else {
          out.push_back(c.l); out.push_back(c.i); out.push_back(c.j); out.push_back(c.k);
        }
      }
    }
  });
  std::vector<int> pstart(part.size() + 1, 0);
  for (size_t c = 0; c < part.size(); ++c) pstart[c + 1] = pstart[c] + (int)part[c].size() / 4;
  const int n = pstart.back();
  H.nleaf = n;
  H.lvl.resize(n); H.ijk.resize(3 * (size_t)n); H.zkey.resize(n);
  pool.run((int)part.size(), [&](int b, int e) {
    for (int c = b; c < e; ++c)
      for (size_t t = 0; 4 * t < part[c].size(); ++t) {
        const int* l = &part[c][4 * t];
        const int q = pstart[c] + (int)t, sh = D - l[0];
        H.lvl[q] = l[0]; H.ijk[3 * q] = l[1]; H.ijk[3 * q + 1] = l[2]; H.ijk[3 * q + 2] = l[3];
        H.zkey[q] = morton3((uint64_t)l[1] << sh, (uint64_t)l[2] << sh, (uint64_t)l[3] << sh);
      }
  });
  // finest-level map: the leaf containing each finest cell
  for (int d = 0; d < 3; ++d) H.nf[d] = cfg.n[d] << D;
  H.fine.resize((size_t)H.nf[0] * H.nf[1] * H.nf[2]);   // every entry is written below
  pool.run(n, [&](int b, int e) {
    for (int q = b; q < e; ++q) {
      const int sh = D - H.lvl[q], w = 1 << sh;
      const size_t i0 = (size_t)H.ijk[3 * q] << sh, j0 = (size_t)H.ijk[3 * q + 1] << sh,
                   k0 = (size_t)H.ijk[3 * q + 2] << sh;
      for (size_t kk = k0; kk < k0 + w; ++kk)
        for (size_t jj = j0; jj < j0 + w; ++jj) {
          int* row = H.fine.data() + (kk * H.nf[1] + jj) * H.nf[0] + i0;
          for (int ii = 0; ii < w; ++ii) row[ii] = q;
        }
    }
  });
  // geometry of every leaf at its own size
  // (every entry is written below; a recycled mesh keeps its capacity)
  H.type.resize(n); H.flags.resize(n); H.S6.resize(6 * (size_t)n);
  H.aw.resize(n); H.nw.resize(3 * (size_t)n); H.rw.resize(3 * (size_t)n);
  H.vbar.resize(n);
  std::atomic<bool> saddle{false}, coarse_cut{false};
  const FarCells far(H, D);
  pool.run(n, [&](int b, int e) {
    for (int q = b; q < e; ++q) {
      CellGeo3 g;
      int A0[3];
      // a leaf of the previous mesh planned at this angle: its geometry
      // is already known (same construction, same inputs)
      const int r = prev ? find_leaf(*prev, D, H.lvl[q], H.ijk[3 * q], H.ijk[3 * q + 1], H.ijk[3 * q + 2]) : -1;
      if (r >= 0) {
        const int sh = D - H.lvl[q];
        for (int d = 0; d < 3; ++d) A0[d] = H.ijk[3 * (size_t)q + d] << sh;
        g.type = prev->type1[r]; g.flags = prev->flags1[r]; g.aw = prev->aw1[r]; g.vbar = prev->vbar1[r];
        for (int f = 0; f < 6; ++f) g.S[f] = prev->S61[6 * (size_t)r + f];
        for (int d = 0; d < 3; ++d) { g.n[d] = prev->nw1[3 * (size_t)r + d]; g.r[d] = prev->r1[3 * (size_t)r + d]; }
      } else {
        leaf_geometry(cfg, H, B, q, g, A0, far);
      }
      if (g.flags & 2) saddle = true;
      if (g.type == TYPE_CUT && H.lvl[q] < D) coarse_cut = true;
      H.type[q] = g.type;
      H.flags[q] = g.flags;
      for (int f = 0; f < 6; ++f) H.S6[6 * q + f] = g.S[f];
      H.aw[q] = g.aw;
      for (int d = 0; d < 3; ++d) {
        H.nw[3 * q + d] = g.n[d];
        H.rw[3 * q + d] = g.aw > 0.0 ? cfg.lo[d] + A0[d] * H.hf[d] + g.r[d] : 0.0;
      }
      H.vbar[q] = g.vbar;
    }
  });
  if (saddle) { err = "a cell is cut twice by the boundary"; return false; }
  if (coarse_cut) { err = "a cut cell above the finest depth (refinement band too narrow)"; return false; }
  // face lists: per leaf, in the order x-, x+, y-, y+, z-, z+, the leaf
  // across (same depth or one coarser), the four of the next finer depth,
  // or the farfield (-1); counted, then written, leaves in parallel
  std::atomic<bool> jump{false};
  auto faces_of = [&](int q, auto&& emit) {
    if (H.type[q] == TYPE_SOLID) return;
    const int l = H.lvl[q];
    for (int t = 0; t < 6; ++t) {
      const double A = H.S6[6 * (size_t)q + t];
      if (A == 0.0) continue;
      const int d = t >> 1, sd = t & 1, d1 = (d + 1) % 3, d2 = (d + 2) % 3;
      int g[3] = {H.ijk[3 * q], H.ijk[3 * q + 1], H.ijk[3 * q + 2]};
      g[d] += sd ? 1 : -1;
      if (g[d] < 0 || g[d] >= (cfg.n[d] << l)) { emit(-1, t, A); continue; }
      const int x = leaf_at(H, D, l, g[0], g[1], g[2]);
      if (H.lvl[x] == l || H.lvl[x] == l - 1) { emit(x, t, A); continue; }
      if (H.lvl[x] < l) { jump = true; continue; }
      for (int b2 = 0; b2 < 2; ++b2)
        for (int b1 = 0; b1 < 2; ++b1) {
          int c[3];
          c[d] = 2 * g[d] + (sd ? 0 : 1); c[d1] = 2 * g[d1] + b1; c[d2] = 2 * g[d2] + b2;
          const int y = find_leaf(H, D, l + 1, c[0], c[1], c[2]);
          if (y < 0) { jump = true; continue; }
          const double Ay = H.S6[6 * (size_t)y + (t ^ 1)];
          if (Ay != 0.0) emit(y, t, Ay);
        }
    }
  };
  // one pass into per-chunk lists (chunks are ranges of leaves, each list
  // sized once for the most entries a chunk can have: 24 per leaf), then
  // concatenated in leaf order
  constexpr int kMaxFaces = 24;
  const size_t nch = (n + HostPool::kChunk - 1) / HostPool::kChunk;
  X.fnb.resize(nch); X.fdir.resize(nch); X.farea.resize(nch);
  std::vector<int>& chunk_faces = X.chunk_faces;
  chunk_faces.resize(nch);
  H.fptr.resize(n + 1);
  H.fptr[0] = 0;
  pool.run(n, [&](int b, int e) {
    const int c = b / HostPool::kChunk;
    const size_t cap = (size_t)kMaxFaces * HostPool::kChunk;
    if (X.fnb[c].size() != cap) { X.fnb[c].resize(cap); X.fdir[c].resize(cap); X.farea[c].resize(cap); }
    int* Fnb = X.fnb[c].data();
    int* Fdir = X.fdir[c].data();
    double* Farea = X.farea[c].data();
    int k = 0;
    for (int q = b; q < e; ++q) {
      const int before = k;
      faces_of(q, [&](int nb, int t, double A) { Fnb[k] = nb; Fdir[k] = t; Farea[k] = A; ++k; });
      H.fptr[q + 1] = k - before;
    }
    chunk_faces[c] = k;
  });
  for (int q = 0; q < n; ++q) H.fptr[q + 1] += H.fptr[q];
  H.nface = H.fptr[n];
  H.fnb.resize(H.nface); H.fdir.resize(H.nface); H.farea.resize(H.nface);
  pool.run((int)nch, [&](int b, int e) {
    for (int c = b; c < e; ++c) {
      const int at = H.fptr[c * HostPool::kChunk], m = chunk_faces[c];
      std::copy(X.fnb[c].begin(), X.fnb[c].begin() + m, H.fnb.begin() + at);
      std::copy(X.fdir[c].begin(), X.fdir[c].begin() + m, H.fdir.begin() + at);
      std::copy(X.farea[c].begin(), X.farea[c].begin() + m, H.farea.begin() + at);
    }
  });
  if (jump) { err = "neighbouring leaves differ by more than one depth"; return false; }
  // masters: centre in gas, else hop across the largest face shared with a
  // leaf of the same depth (order x+, x-, y+, y-, z+, z-), at most 4 hops
  H.master.resize(n);
  const int dir_order[6] = {1, 0, 3, 2, 5, 4};
  std::atomic<bool> master_bad{false};
  pool.run(n, [&](int qb, int qe) {
  for (int q = qb; q < qe; ++q) {
    H.master[q] = -1;
    if (H.type[q] == TYPE_SOLID) continue;
    int cur = q, hops = 0, seen[5] = {q, -1, -1, -1, -1};
    bool ok = true;
    while (!(H.flags[cur] & 1)) {
      const int l = H.lvl[cur];
      double L[6];
      int nb[6];
      for (int u = 0; u < 6; ++u) {
        const int t = dir_order[u], d = t >> 1;
        int g[3] = {H.ijk[3 * cur], H.ijk[3 * cur + 1], H.ijk[3 * cur + 2]};
        g[d] += (t & 1) ? 1 : -1;
        L[u] = 0.0; nb[u] = -1;
        if (g[d] < 0 || g[d] >= (cfg.n[d] << l)) continue;
        nb[u] = find_leaf(H, D, l, g[0], g[1], g[2]);
        L[u] = H.S6[6 * (size_t)cur + t];
      }
      double M = 0.0;
      for (int u = 0; u < 6; ++u) M = std::max(M, L[u]);
      if (!(M > 0.0) || hops == 4) { ok = false; break; }
      const double tie = M * (1.0 - 1e-12);
      int u = 0;
      while (L[u] < tie) ++u;
      if (nb[u] < 0) { ok = false; break; }
      cur = nb[u];
      ++hops;
      for (int h = 0; h < hops; ++h) if (seen[h] == cur) ok = false;
      if (!ok) break;
      seen[hops] = cur;
    }
    if (!ok) { master_bad = true; continue; }
    H.master[q] = cur;
  }
  });
  if (master_bad) { err = "master search cycles, leaves the domain, crosses a change of depth or needs more than 4 hops"; return false; }
  std::atomic<bool> not_own{false};
  pool.run(n, [&](int b, int e) {
    for (int q = b; q < e; ++q)
      if (H.master[q] >= 0 && H.master[H.master[q]] != H.master[q]) not_own = true;
  });
  if (not_own) { err = "a master is not its own master"; return false; }
  if (!order_cvs(H, nullptr, err)) return false;
  // control-volume volumes (members in order) and the counts, per chunk
  H.vcv.resize(n);
  pool.run(n, [&](int b, int e) { std::fill(H.vcv.begin() + b, H.vcv.begin() + e, 0.0); });
  const int ncv = (int)H.cv.size();
  std::vector<int>& cnt3 = X.counts;
  cnt3.assign(3 * (size_t)((std::max(ncv, n) + HostPool::kChunk - 1) / HostPool::kChunk), 0);
  pool.run(ncv, [&](int b, int e) {
    int irr = 0, mem = 0;
    for (int s = b; s < e; ++s) {
      double v = 0.0;
      bool wall = false;
      for (int k = H.cvptr[s]; k < H.cvptr[s + 1]; ++k) {
        v += H.vbar[H.cvmem[k]];
        wall = wall || H.aw[H.cvmem[k]] > 0.0;
      }
      H.vcv[H.cv[s]] = v;
      const int nm = H.cvptr[s + 1] - H.cvptr[s];
      irr += nm > 1 || wall;
      mem += nm - 1;
    }
    cnt3[3 * (size_t)(b / HostPool::kChunk)] = irr;
    cnt3[3 * (size_t)(b / HostPool::kChunk) + 1] = mem;
  });
  pool.run(n, [&](int b, int e) {
    int sol = 0;
    for (int q = b; q < e; ++q) sol += H.type[q] == TYPE_SOLID;
    cnt3[3 * (size_t)(b / HostPool::kChunk) + 2] = sol;
  });
  H.n_irr = 0; H.n_members = 0; H.n_solid = 0;
  for (size_t c = 0; 3 * c < cnt3.size(); ++c) {
    H.n_irr += cnt3[3 * c]; H.n_members += cnt3[3 * c + 1]; H.n_solid += cnt3[3 * c + 2];
  }
  // the plan arrays (type1 .. rmem) keep their stale contents and sizes: the
  // plan of a step writes every entry, and resizing a recycled mesh's arrays
  // to about the same size then costs no fill
  return true;
}

// Turning body, the step from t^n to t^{n+1} on the mesh H of t^n
// (Section 5, steps 3 and 7): the leaves' types and gas volumes with the
// body at th1; the control volume of t^n each leaf receives from (its
// master; a leaf solid at t^n and not at t^{n+1} hops across its largest
// face at t^{n+1} to a leaf of the same depth, order x+, x-, y+, y-, z+,
// z-, at most 4 hops, and takes that leaf's control volume); each control
// volume's volume at t^{n+1} (the sum over its receivers, leaf order) and
// its receivers (not solid at t^{n+1}).  Control volumes whose volume or
// receivers change are ordered with the cut ones.
bool plan_amr_move(const cc_config& cfg, const cc_body& body, double th1, AmrHost& H, std::string& err) {
  const int n = H.nleaf, D = cfg.amr_depth;
  const BodyDev B = body_at(body, th1);
  H.type1.resize(n); H.vbar1.resize(n); H.flags1.resize(n); H.S61.resize(6 * (size_t)n);
  H.aw1.resize(n); H.nw1.resize(3 * (size_t)n); H.r1.resize(3 * (size_t)n);
  std::vector<double>& S61 = H.S61;
  std::atomic<bool> saddle{false}, coarse_cut{false};
  const FarCells far(H, D);
  HostPool::get().run(n, [&](int b, int e) {
    for (int q = b; q < e; ++q) {
      CellGeo3 g;
      int A0[3];
      leaf_geometry(cfg, H, B, q, g, A0, far);
      if (g.flags & 2) saddle = true;
      if (g.type == TYPE_CUT && H.lvl[q] < D) coarse_cut = true;
      H.type1[q] = g.type;
      H.vbar1[q] = g.vbar;
      H.flags1[q] = g.flags;
      H.aw1[q] = g.aw;
      for (int f = 0; f < 6; ++f) S61[6 * (size_t)q + f] = g.S[f];
      for (int d = 0; d < 3; ++d) { H.nw1[3 * (size_t)q + d] = g.n[d]; H.r1[3 * (size_t)q + d] = g.r[d]; }
    }
  });
  if (saddle) { err = "a cell is cut twice by the boundary at the next time"; return false; }
  if (coarse_cut) { err = "the body moved out of the refined band within one step"; return false; }
  std::vector<int> target(H.master);
  const int dir_order[6] = {1, 0, 3, 2, 5, 4};
  for (int q = 0; q < n; ++q) {
    if (!(H.type[q] == TYPE_SOLID && H.type1[q] != TYPE_SOLID)) continue;
    int cur = q, hops = 0;
    while (H.master[cur] < 0 && hops < 4) {
      const int l = H.lvl[cur];
      double L[6], M = 0.0;
      int nb[6];
      for (int u = 0; u < 6; ++u) {
        const int t = dir_order[u], d = t >> 1;
        int g[3] = {H.ijk[3 * cur], H.ijk[3 * cur + 1], H.ijk[3 * cur + 2]};
        g[d] += (t & 1) ? 1 : -1;
        nb[u] = -1; L[u] = 0.0;
        if (g[d] < 0 || g[d] >= (cfg.n[d] << l)) continue;
        nb[u] = find_leaf(H, D, l, g[0], g[1], g[2]);
        L[u] = S61[6 * (size_t)cur + t];
        M = std::max(M, L[u]);
      }
      if (!(M > 0.0)) break;
      const double tie = M * (1.0 - 1e-12);
      int u = 0;
      while (L[u] < tie) ++u;
      if (nb[u] < 0) break;
      cur = nb[u];
      ++hops;
    }
    if (H.master[cur] < 0) { err = "a leaf appearing at the next time found no control volume"; return false; }
    target[q] = H.master[cur];
  }
  H.vnew.assign(n, 0.0);
  std::vector<int> rcnt(n, 0);
  for (int q = 0; q < n; ++q)
    if (target[q] >= 0) {
      H.vnew[target[q]] += H.vbar1[q];
      if (H.type1[q] != TYPE_SOLID) rcnt[target[q]]++;
    }
  // receivers grouped by master (leaf order), compared with the members
  std::vector<int> rstart(n + 1, 0);
  for (int q = 0; q < n; ++q) rstart[q + 1] = rstart[q] + rcnt[q];
  std::vector<int> rlist(rstart[n]), fill(n, 0);
  for (int q = 0; q < n; ++q)
    if (target[q] >= 0 && H.type1[q] != TYPE_SOLID) rlist[rstart[target[q]] + fill[target[q]]++] = q;
  std::vector<char> changed(n, 0);
  for (size_t s = 0; s < H.cv.size(); ++s) {
    const int m = H.cv[s];
    const int nm = H.cvptr[s + 1] - H.cvptr[s];
    bool same = H.vnew[m] == H.vcv[m] && rcnt[m] == nm;
    for (int e = 0; same && e < nm; ++e) same = rlist[rstart[m] + e] == H.cvmem[H.cvptr[s] + e];
    changed[m] = !same;
  }
  if (!order_cvs(H, &changed, err)) return false;
  H.rptr.assign(H.cv.size() + 1, 0);
  H.rmem.clear();
  for (size_t s = 0; s < H.cv.size(); ++s) {
    const int m = H.cv[s];
    for (int e = rstart[m]; e < rstart[m + 1]; ++e) H.rmem.push_back(rlist[e]);
    H.rptr[s + 1] = (int)H.rmem.size();
  }
  return true;
}

// The state carried from the mesh of t^n (old, with its leaves' gas volumes
// at t^{n+1}) to the mesh of t^{n+1} (Section 5.1, mesh adaptation): a leaf
// that is also an old leaf, or lies inside one, takes its value (0th-order
// prolongation); a leaf that covers old leaves takes their gas-volume
// weighted mean (restriction), summed in old-leaf order; solid leaves are 0.
// The old leaves inside a leaf are a contiguous range of the Z-order.
void build_amr_remap(const AmrHost& O, const AmrHost& H, int depth, AmrRemap& R) {
  const int n = H.nleaf;
  R.sptr.assign(n + 1, 0);
  // entries of each chunk of new leaves (chunks are leaf ranges), then
  // concatenated in leaf order
  struct Chunk { std::vector<int> src; std::vector<double> wgt; };
  std::vector<Chunk> ch((n + HostPool::kChunk - 1) / HostPool::kChunk);
  HostPool& pool = HostPool::get();
  pool.run(n, [&](int b, int e) {
    Chunk& C = ch[b / HostPool::kChunk];
    for (int q = b; q < e; ++q) {
      const size_t before = C.src.size();
      if (H.type[q] != TYPE_SOLID) {
        const int l = H.lvl[q], i = H.ijk[3 * q], j = H.ijk[3 * q + 1], k = H.ijk[3 * q + 2];
        // the old leaf at this leaf's corner: the same leaf or one containing it
        const int s = leaf_at(O, depth, l, i, j, k);
        if (O.lvl[s] <= l) {
          C.src.push_back(s); C.wgt.push_back(1.0);
        } else {
          const int sh = depth - l;
          const uint64_t z0 = morton3((uint64_t)i << sh, (uint64_t)j << sh, (uint64_t)k << sh),
                         z1 = z0 + (1ULL << (3 * sh));
          for (size_t r = std::lower_bound(O.zkey.begin(), O.zkey.end(), z0) - O.zkey.begin();
               r < O.zkey.size() && O.zkey[r] < z1; ++r) {
            C.src.push_back((int)r);
            C.wgt.push_back(O.vbar1[r]);
          }
        }
      }
      R.sptr[q + 1] = (int)(C.src.size() - before);
    }
  });
  for (int q = 0; q < n; ++q) R.sptr[q + 1] += R.sptr[q];
  R.src.resize(R.sptr[n]); R.wgt.resize(R.sptr[n]);
  pool.run((int)ch.size(), [&](int b, int e) {
    for (int c = b; c < e; ++c) {
      const int at = R.sptr[c * HostPool::kChunk];
      std::copy(ch[c].src.begin(), ch[c].src.end(), R.src.begin() + at);
      std::copy(ch[c].wgt.begin(), ch[c].wgt.end(), R.wgt.begin() + at);
    }
  });
}

// ---------------------------------------------------------------------
// device
// ---------------------------------------------------------------------
namespace {

constexpr int kWaveA = 64;
constexpr int kAmrRC = 4;    // velocities per lane and pass of the general octree step
constexpr int kAmrRCS = 2;   // velocities per lane and pass of the streaming octree step
constexpr int kAmrPipe = 2;  // streaming octree step: passes of loads issued ahead of the computed one
constexpr int kAmrFU = 2;    // general octree step: faces whose loads are requested together

__device__ inline double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWaveA);
  return v;
}

__device__ inline double vnodeA(double vmin, double dv, int i) { return vmin + (i + 0.5) * dv; }

struct AmrArgs {
  const double* in;
  double* out;
  AmrDev G;
  double* mom;        // 8 per leaf: A, ux, uy, uz, 1/(2T), dt/tau, rho, -
  double* part;       // 4 per block: wall force and mass of the state at t^n
  int per_simple, per, per_irr;   // blocks per XCD of the three kinds of control volumes
  double vmin, dv, w, dt, tau_coef, t_wall;
  double om, cx, cy;              // turning body: angular velocity at t^n, axis (z) position
  int w0;                         // first control volume of the moment pass
};

// record of the relaxation from the moment sums of one control volume
__device__ inline void write_record(double* mom, const int* mem, int nm, const double s[5],
                                    double w, double dt, double tau_coef) {
  const double rho = s[0] * w;
  const double ux = s[1] * w / rho, uy = s[2] * w / rho, uz = s[3] * w / rho;
  const double en = 0.5 * s[4] * w;
  const double T = (2.0 * en / rho - (ux * ux + uy * uy + uz * uz)) / 3.0;
  const double rec[8] = {rho / pow(2.0 * M_PI * T, 1.5), ux, uy, uz, 0.5 / T,
                         tau_coef > 0.0 ? dt * rho / tau_coef : 0.0, rho, 0.0};
  for (int t = 0; t < nm; ++t)
    for (int q = 0; q < 8; ++q) mom[8 * (size_t)mem[t] + q] = rec[q];
}

// IRR = false: control volumes [nsimple, nreg) (one member, no wall face,
// a finer neighbour on some face); IRR = true: [nreg, ncv) (cut or merged).
// These are few, so each gets a 256-thread block (one wave each would leave
// most of the GPU waiting on memory); the four waves split the velocities.
// MV (with IRR): turning body.  The walls move with om e_z x (r - axis):
// wall density, wall flux and stress use v - u_w; the update carries the
// ratio V^n / V^{n+1,*} of eq. (eq-schema3D) and goes to the control
// volume's receivers at t^{n+1}; the partials hold the torque about the
// axis in place of Fz.
template <int N, bool IRR, bool MV = false>
__global__ void __launch_bounds__(256) k_amr_step(AmrArgs A) {
  constexpr int NV = N * N * N;
  constexpr int NT = 256;
  constexpr int R = (NV + NT - 1) / NT;                      // velocities per thread
  constexpr int RC = R < kAmrRC ? R : kAmrRC;   // per pass
  constexpr int NP = (R + RC - 1) / RC;
  __shared__ double lds[4][2];
  // XCD-aware order: block b runs on XCD b % 8, and the blocks of one XCD
  // take a contiguous range of control volumes (neighbours in Z-order share
  // that XCD's L2)
  const int per = IRR ? A.per_irr : A.per;
  const int w0 = IRR ? A.G.nreg : A.G.nsimple, ncv = IRR ? A.G.ncv - A.G.nreg : A.G.nreg - A.G.nsimple;
  const int blk = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (blk >= ncv) return;    // uniform over the block
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const AmrDev& G = A.G;
  const int w = w0 + blk;
  const int m = G.cv[w], b = G.cvptr[w], nm = G.cvptr[w + 1] - b;
  const double* rec = A.mom + 8 * (size_t)m;
  const double Am = rec[0], ux = rec[1], uy = rec[2], uz = rec[3], inv2T = rec[4], dtau = rec[5];
  const double mass_n = G.vcv[m] * rec[6];   // before the record is overwritten
  const double dtV = A.dt / G.vcv[m];
  const double vn = MV ? G.vnew[m] : 0.0;
  const double ratio = MV && vn > 0.0 ? G.vcv[m] / vn : 1.0;
  const double dtVn = MV ? (vn > 0.0 ? A.dt / vn : 0.0) : dtV;
  const double* own = A.in + (size_t)m * NV;
  // block sum (waves added in order); every thread gets the total
  auto bsum = [&](double v) {
    v = wsum(v);
    __syncthreads();
    if (lane == 0) lds[wave][0] = v;
    __syncthreads();
    return ((lds[0][0] + lds[1][0]) + lds[2][0]) + lds[3][0];
  };
  double tx = 0.0, ty = 0.0, tz = 0.0;   // per-axis factors of the Maxwellian, in every wave
  if (lane < N) {
    const double v = vnodeA(A.vmin, A.dv, lane);
    tx = exp(-(v - ux) * (v - ux) * inv2T);
    ty = exp(-(v - uy) * (v - uy) * inv2T);
    tz = exp(-(v - uz) * (v - uz) * inv2T);
  }
  // wall density of each member with a wall face (zero net mass flux)
  const double Tw = A.t_wall, cw = 1.0 / pow(2.0 * M_PI * Tw, 1.5), i2Tw = 0.5 / Tw;
  double phiw[IRR ? kMaxMembers : 1];
  double uwx[MV ? kMaxMembers : 1], uwy[MV ? kMaxMembers : 1];
  bool any_wall = false;
  // the control volume's values of the thread's velocities, requested
  // together (no per-lane condition), for the wall densities
  double fw0[IRR ? R : 1];
  if (IRR) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int p = i * NT + tid;
      fw0[i] = own[p < NV ? p : 0];
    }
  }
  for (int t = 0; t < (IRR ? nm : 0); ++t) {
    const int k = G.cvmem[b + t];
    phiw[t] = 0.0;
    if (MV) { uwx[t] = 0.0; uwy[t] = 0.0; }
    if (!(G.aw[k] > 0.0)) continue;
    any_wall = true;
    const double n0 = G.nw[3 * k], n1 = G.nw[3 * k + 1], n2 = G.nw[3 * k + 2];
    if (MV) {
      uwx[t] = -A.om * (G.rw[3 * k + 1] - A.cy);
      uwy[t] = A.om * (G.rw[3 * k] - A.cx);
    }
    const double ux_ = MV ? uwx[t] : 0.0, uy_ = MV ? uwy[t] : 0.0;
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int i = 0; i < (IRR ? R : 1); ++i) {
      const int p = i * NT + tid;
      if (p >= NV) continue;
      const double vx = vnodeA(A.vmin, A.dv, p % N) - ux_, vy = vnodeA(A.vmin, A.dv, (p / N) % N) - uy_,
                   vz = vnodeA(A.vmin, A.dv, p / (N * N));
      const double cn = vx * n0 + vy * n1 + vz * n2;
      if (cn > 0.0) num += cn * fw0[i];
      else if (cn < 0.0) den += cn * cw * exp(-(vx * vx + vy * vy + vz * vz) * i2Tw);
    }
    num = bsum(num);
    den = bsum(den);
    phiw[t] = den != 0.0 ? -num / den : 0.0;
  }
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double fx = 0.0, fy = 0.0, fz = 0.0;   // MV: fz holds the torque about the axis
  for (int pass = 0; pass < NP; ++pass) {
    // the thread id is laundered per pass so that the velocity constants of
    // a pass are recomputed where used instead of being held across passes
    int lv = tid;
    asm volatile("" : "+v"(lv));
    double fo[RC], acc[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      const int p = (pass * RC + r) * NT + lv;
      fo[r] = p < NV ? own[p] : 0.0;
      acc[r] = 0.0;
    }
    for (int t = 0; t < (IRR ? nm : 1); ++t) {
      const int k = IRR ? G.cvmem[b + t] : m;
      if constexpr (IRR) {
        // the cut kernels take the faces one by one: their registers decide
        // how many of their blocks fit beside the streaming kernel
        for (int e = G.fptr[k]; e < G.fptr[k + 1]; ++e) {
          const int nb = G.fnb[e], dir = G.fdir[e];
          const double area = G.farea[e];
          const double* nrow = nb >= 0 ? A.in + (size_t)nb * NV : G.ghost;
          const double sg = (dir & 1) ? 1.0 : -1.0;
          // the face's axis is uniform over the block: one loop per axis
          auto gather = [&](auto comp) {
#pragma unroll
            for (int r = 0; r < RC; ++r) {
              const int p = (pass * RC + r) * NT + lv;
              const double c = sg * vnodeA(A.vmin, A.dv, comp(p));   // outward normal velocity
              const double fn = nrow[p < NV ? p : 0];   // no per-lane condition on the load
              acc[r] += area * (fmax(c, 0.0) * fo[r] + fmin(c, 0.0) * fn);
            }
          };
          switch (dir >> 1) {
            case 0: gather([](int p) { return p % N; }); break;
            case 1: gather([](int p) { return (p / N) % N; }); break;
            default: gather([](int p) { return p / (N * N); }); break;
          }
        }
      } else {
        // faces in groups of kAmrFU, the group's loads requested together;
        // a lane whose velocity leaves through a face (or lies past the last
        // velocity) reads its own value there, already in the cache, and
        // the group's missing faces have zero area
        constexpr int FU = kAmrFU;
        const int e0 = G.fptr[k], e1 = G.fptr[k + 1];
        for (int e = e0; e < e1; e += FU) {
          const double* nrow[FU];
          double area[FU], sg[FU];
          int ax[FU];
#pragma unroll
          for (int j = 0; j < FU; ++j) {
            const bool ok = e + j < e1;
            const int ej = ok ? e + j : e;
            const int nb = G.fnb[ej], dir = G.fdir[ej];
            area[j] = ok ? G.farea[ej] : 0.0;
            nrow[j] = nb >= 0 ? A.in + (size_t)nb * NV : G.ghost;
            sg[j] = (dir & 1) ? 1.0 : -1.0;
            ax[j] = dir >> 1;
          }
          double c[FU][RC], fn[FU][RC];
#pragma unroll
          for (int j = 0; j < FU; ++j)
#pragma unroll
            for (int r = 0; r < RC; ++r) {
              const int p0 = (pass * RC + r) * NT + lv;
              const int p = p0 < NV ? p0 : 0;
              const int pa = ax[j] == 0 ? p % N : (ax[j] == 1 ? (p / N) % N : p / (N * N));
              c[j][r] = sg[j] * vnodeA(A.vmin, A.dv, pa);   // outward normal velocity
              fn[j][r] = (c[j][r] < 0.0 && p0 < NV ? nrow[j] : own)[p];
            }
#pragma unroll
          for (int j = 0; j < FU; ++j)
#pragma unroll
            for (int r = 0; r < RC; ++r)
              acc[r] += area[j] * (fmax(c[j][r], 0.0) * fo[r] + fmin(c[j][r], 0.0) * fn[j][r]);
        }
      }
      if (IRR && any_wall && G.aw[k] > 0.0) {
        const double awk = G.aw[k], n0 = G.nw[3 * k], n1 = G.nw[3 * k + 1], n2 = G.nw[3 * k + 2];
        const double ux_ = MV ? uwx[t] : 0.0, uy_ = MV ? uwy[t] : 0.0;
        const double lx = MV ? G.rw[3 * k] - A.cx : 0.0, ly = MV ? G.rw[3 * k + 1] - A.cy : 0.0;
#pragma unroll
        for (int r = 0; r < RC; ++r) {
          const int p = (pass * RC + r) * NT + lv;
          if (p >= NV) continue;
          // velocity relative to the wall
          const double vx = vnodeA(A.vmin, A.dv, p % N) - ux_, vy = vnodeA(A.vmin, A.dv, (p / N) % N) - uy_,
                       vz = vnodeA(A.vmin, A.dv, p / (N * N));
          const double cn = vx * n0 + vy * n1 + vz * n2;
          const double fw = phiw[t] * cw * exp(-(vx * vx + vy * vy + vz * vz) * i2Tw);
          acc[r] += awk * (fmin(cn, 0.0) * fw + fmax(cn, 0.0) * fo[r]);
          const double fv = cn < 0.0 ? fw : (cn > 0.0 ? fo[r] : 0.0);
          fx += awk * vx * cn * fv; fy += awk * vy * cn * fv;
          if (MV) fz += awk * (lx * vy - ly * vx) * cn * fv;
          else fz += awk * vz * cn * fv;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      const int p = (pass * RC + r) * NT + lv;
      if (p >= NV) continue;
      const int p1 = p % N, p2 = (p / N) % N, p3 = p / (N * N);
      const double E = Am * __shfl(tx, p1, kWaveA) * __shfl(ty, p2, kWaveA) * __shfl(tz, p3, kWaveA);
      const double f = fo[r];
      const double fn = MV ? ratio * f - dtVn * acc[r] + ratio * dtau * (E - f) : f - dtV * acc[r] + dtau * (E - f);
      if (MV)
        for (int e = G.rptr[w]; e < G.rptr[w + 1]; ++e) A.out[(size_t)G.rmem[e] * NV + p] = fn;
      else if (IRR)
        for (int t = 0; t < nm; ++t) A.out[(size_t)G.cvmem[b + t] * NV + p] = fn;
      else
        A.out[(size_t)m * NV + p] = fn;
      const double vx = vnodeA(A.vmin, A.dv, p1), vy = vnodeA(A.vmin, A.dv, p2), vz = vnodeA(A.vmin, A.dv, p3);
      s[0] += fn; s[1] += vx * fn; s[2] += vy * fn; s[3] += vz * fn;
      s[4] += (vx * vx + vy * vy + vz * vz) * fn;
    }
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) s[q] = bsum(s[q]);
  if (IRR && any_wall) { fx = bsum(fx); fy = bsum(fy); fz = bsum(fz); }
  if (tid == 0) {
    if (!MV) write_record(A.mom, G.cvmem + b, nm, s, A.w, A.dt, A.tau_coef);
    // partials after the streaming kernel's blocks: one per control volume
    const size_t slot = (size_t)(A.G.nsimple + 3) / 4 + (IRR ? A.G.nreg - A.G.nsimple : 0) + blk;
    A.part[4 * slot + 0] = IRR ? fx * A.w : 0.0;
    A.part[4 * slot + 1] = IRR ? fy * A.w : 0.0;
    A.part[4 * slot + 2] = IRR ? fz * A.w : 0.0;
    A.part[4 * slot + 3] = mass_n;
  }
}

// Control volumes [0, nsimple): gas leaves with one neighbour (or the
// farfield) per face direction.  The upwind flux of an axis is then
// A |v| (f - f_up) with f_up from the face's leaf on the upwind side, so
// each velocity needs its own value and three upwind values, all
// independent loads.
template <int N>
__global__ void __launch_bounds__(256) k_amr_simple(AmrArgs A) {
  constexpr int NV = N * N * N;
  constexpr int R = (NV + kWaveA - 1) / kWaveA;
  constexpr int RC = R < kAmrRCS ? R : kAmrRCS;
  constexpr int NP = (R + RC - 1) / RC;
  __shared__ double lds[4][4];
  const int per = A.per_simple, ncv = A.G.nsimple;
  const int blk = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int w = blk * 4 + wave;
  if (blk * 4 >= ncv) return;    // uniform over the block
  const bool live = w < ncv;
  const AmrDev& G = A.G;
  const int m = live ? G.cv[w] : 0;
  const double* rec = A.mom + 8 * (size_t)m;
  const double Am = rec[0], ux = rec[1], uy = rec[2], uz = rec[3], inv2T = rec[4], dtau = rec[5];
  const double mass_n = live ? G.vcv[m] * rec[6] : 0.0;
  const double dtV = A.dt / G.vcv[m];
  const double* own = A.in + (size_t)m * NV;
  const int e0 = G.fptr[m];
  const double* row[6];
  double ar[6];
  for (int t = 0; t < 6; ++t) {
    const int nb = live ? G.fnb[e0 + t] : -1;
    row[t] = nb >= 0 ? A.in + (size_t)nb * NV : G.ghost;
    ar[t] = live ? G.farea[e0 + t] : 0.0;
  }
  double tx = 0.0, ty = 0.0, tz = 0.0;
  if (lane < N) {
    const double v = vnodeA(A.vmin, A.dv, lane);
    tx = exp(-(v - ux) * (v - ux) * inv2T);
    ty = exp(-(v - uy) * (v - uy) * inv2T);
    tz = exp(-(v - uz) * (v - uz) * inv2T);
  }
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  // passes of RC velocities per lane; the loads of pass k + kAmrPipe
  // are issued before pass k is computed (kAmrPipe + 1 stages)
  constexpr int ST = kAmrPipe + 1;
  double fo[ST][RC], fx[ST][RC], fy[ST][RC], fz[ST][RC];
  // Every lane issues every load (lanes past the last velocity read the
  // first one; their values are not used), and the whole pipeline sits
  // under one branch on the wave, so that no branch splits the loads and
  // the compiler waits for each pass's loads only, not for the whole
  // window.  in_v is decided from the plain lane id, so that it folds to
  // true where NV is a multiple of the wave.
  auto in_v = [&](int pass, int r) { return (pass * RC + r) * kWaveA + lane < NV; };
  auto load = [&](int pass, int st) {
    // the lane id is laundered per pass so that the velocity constants of a
    // pass are recomputed where used instead of being held across passes
    int lv = lane;
    asm volatile("" : "+v"(lv));
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      const int p0 = (pass * RC + r) * kWaveA + lv;
      const int p = in_v(pass, r) ? p0 : lv;
      const int p1 = p % N, p2 = (p / N) % N, p3 = p / (N * N);
      // upwind side: the x- face's leaf for v_x > 0, the x+ face's for v_x < 0
      const bool px = vnodeA(A.vmin, A.dv, p1) > 0.0, py = vnodeA(A.vmin, A.dv, p2) > 0.0,
                 pz = vnodeA(A.vmin, A.dv, p3) > 0.0;
      fo[st][r] = own[p];
      fx[st][r] = (px ? row[0] : row[1])[p];
      fy[st][r] = (py ? row[2] : row[3])[p];
      fz[st][r] = (pz ? row[4] : row[5])[p];
    }
  };
  if (live) {
#pragma unroll
    for (int k = 0; k < ST - 1 && k < NP; ++k) load(k, k);
#pragma unroll
    for (int pass = 0; pass < NP; ++pass) {
      const int st = pass % ST;
      if (ST > 1 && pass + ST - 1 < NP) load(pass + ST - 1, (pass + ST - 1) % ST);
      int lv = lane;
      asm volatile("" : "+v"(lv));
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        const bool in = in_v(pass, r);
        const int p0 = (pass * RC + r) * kWaveA + lv;
        const int p = in ? p0 : lv;
        const int p1 = p % N, p2 = (p / N) % N, p3 = p / (N * N);
        const double vx = vnodeA(A.vmin, A.dv, p1), vy = vnodeA(A.vmin, A.dv, p2), vz = vnodeA(A.vmin, A.dv, p3);
        const double f = fo[st][r];
        const double acc = (vx > 0.0 ? ar[0] : ar[1]) * fabs(vx) * (f - fx[st][r]) +
                           (vy > 0.0 ? ar[2] : ar[3]) * fabs(vy) * (f - fy[st][r]) +
                           (vz > 0.0 ? ar[4] : ar[5]) * fabs(vz) * (f - fz[st][r]);
        const double E = Am * __shfl(tx, p1, kWaveA) * __shfl(ty, p2, kWaveA) * __shfl(tz, p3, kWaveA);
        const double fn = f - dtV * acc + dtau * (E - f);
        if (in) A.out[(size_t)m * NV + p] = fn;
        const double fv = in ? fn : 0.0;
        s[0] += fv; s[1] += vx * fv; s[2] += vy * fv; s[3] += vz * fv;
        s[4] += (vx * vx + vy * vy + vz * vz) * fv;
      }
      if (ST == 1 && pass + 1 < NP) load(pass + 1, 0);
    }
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) s[q] = wsum(s[q]);
  if (lane == 0) {
    if (live) write_record(A.mom, &G.cv[w], 1, s, A.w, A.dt, A.tau_coef);
    lds[wave][0] = 0.0; lds[wave][1] = 0.0; lds[wave][2] = 0.0; lds[wave][3] = mass_n;
  }
  __syncthreads();
  if (threadIdx.x < 4)
    A.part[4 * (size_t)blk + threadIdx.x] =
        ((lds[0][threadIdx.x] + lds[1][threadIdx.x]) + lds[2][threadIdx.x]) + lds[3][threadIdx.x];
}

// record of every control volume from its current value (one wave each)
template <int N>
__global__ void __launch_bounds__(256) k_amr_mom(AmrArgs A) {
  constexpr int NV = N * N * N;
  const int w = A.w0 + blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (w >= A.G.ncv) return;
  const int m = A.G.cv[w], b = A.G.cvptr[w], nm = A.G.cvptr[w + 1] - b;
  const double* own = A.in + (size_t)m * NV;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int p = lane; p < NV; p += kWaveA) {
    const double vx = vnodeA(A.vmin, A.dv, p % N), vy = vnodeA(A.vmin, A.dv, (p / N) % N),
                 vz = vnodeA(A.vmin, A.dv, p / (N * N));
    const double f = own[p];
    s[0] += f; s[1] += vx * f; s[2] += vy * f; s[3] += vz * f;
    s[4] += (vx * vx + vy * vy + vz * vz) * f;
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) s[q] = wsum(s[q]);
  if (lane == 0) write_record(A.mom, A.G.cvmem + b, nm, s, A.w, A.dt, A.tau_coef);
}

// merge of the control volumes with several members: value = sum_k V_k F_k / V
__global__ void __launch_bounds__(256) k_amr_merge(AmrDev G, double* __restrict__ st, int nvel, int w0) {
  const int w = w0 + blockIdx.x;
  const int m = G.cv[w], b = G.cvptr[w], nm = G.cvptr[w + 1] - b;
  if (nm <= 1) return;
  for (int p = threadIdx.x; p < nvel; p += blockDim.x) {
    double acc = 0.0;
    for (int t = 0; t < nm; ++t) {
      const int k = G.cvmem[b + t];
      acc += G.vbar[k] * st[(size_t)k * nvel + p];
    }
    const double v = acc / G.vcv[m];
    for (int t = 0; t < nm; ++t) st[(size_t)G.cvmem[b + t] * nvel + p] = v;
  }
}

__global__ void k_amr_init(AmrDev G, double* __restrict__ st, int nvel, int load, const double* __restrict__ f) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)G.nleaf * nvel) return;
  const int c = (int)(t / nvel), p = (int)(t % nvel);
  st[t] = G.type[c] == TYPE_SOLID ? 0.0 : (load ? f[t] : G.ghost[p]);
}

__global__ void k_amr_tables(AmrDev G, int N, double vmin, double dv, double rho, double ux, double uy,
                             double uz, double T) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N * N * N) return;
  const double vx = vmin + (p % N + 0.5) * dv, vy = vmin + ((p / N) % N + 0.5) * dv,
               vz = vmin + (p / (N * N) + 0.5) * dv;
  const double cx = vx - ux, cy = vy - uy, cz = vz - uz;
  G.ghost[p] = rho / pow(2.0 * M_PI * T, 1.5) * exp(-(cx * cx + cy * cy + cz * cz) / (2.0 * T));
}

// diag row from the block partials of the step (fixed order)
__global__ void __launch_bounds__(1024) k_amr_reduce(const double* __restrict__ part, int nblk,
                                                    double* __restrict__ row) {
  __shared__ double lds[16][4];
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int t = threadIdx.x; t < nblk; t += blockDim.x)
    for (int q = 0; q < 4; ++q) a[q] += part[4 * (size_t)t + q];
  for (int q = 0; q < 4; ++q) a[q] = wsum(a[q]);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < 4; ++q) lds[wave][q] = a[q];
  __syncthreads();
  if (threadIdx.x < 4) {
    double r = 0.0;
    for (int v = 0; v < 16; ++v) r += lds[v][threadIdx.x];
    row[threadIdx.x] = r;
  }
}

// state carried to the next mesh: new leaf q takes
// sum_e wgt[e] F[src[e]] / sum_e wgt[e] (0 with no entry); one block per
// leaf, its threads over the velocities (the entries are uniform over the
// block).  The moment sums of the new value give the leaf's relaxation
// record (that of its control volume when it is the only member; the
// moment pass redoes the control volumes with several members after their
// merge).
template <int N>
__global__ void __launch_bounds__(256) k_amr_remap(const int* __restrict__ sptr, const int* __restrict__ src,
                                                  const double* __restrict__ wgt, const double* __restrict__ from,
                                                  double* __restrict__ to, AmrArgs A) {
  constexpr int NV = N * N * N;
  __shared__ double lds[4][5];
  const int q = blockIdx.x;
  const int e0 = sptr[q], e1 = sptr[q + 1];
  double* dst = to + (size_t)q * NV;
  const bool copy = e1 - e0 == 1 && wgt[e0] == 1.0;   // the same leaf, or one containing it
  double W = 0.0;
  for (int e = e0; e < e1; ++e) W += wgt[e];
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int p = threadIdx.x; p < NV; p += 256) {
    double v;
    if (copy) {
      v = 0.0 + 1.0 * from[(size_t)src[e0] * NV + p];
    } else {
      double acc = 0.0;
      for (int e = e0; e < e1; ++e) acc += wgt[e] * from[(size_t)src[e] * NV + p];
      v = W > 0.0 ? acc / W : 0.0;
    }
    dst[p] = v;
    const double vx = vnodeA(A.vmin, A.dv, p % N), vy = vnodeA(A.vmin, A.dv, (p / N) % N),
                 vz = vnodeA(A.vmin, A.dv, p / (N * N));
    s[0] += v; s[1] += vx * v; s[2] += vy * v; s[3] += vz * v;
    s[4] += (vx * vx + vy * vy + vz * vz) * v;
  }
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double t = wsum(s[k]);
    if ((threadIdx.x & 63) == 0) lds[wave][k] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0 && W > 0.0) {
    double t[5];
    for (int k = 0; k < 5; ++k) t[k] = ((lds[0][k] + lds[1][k]) + lds[2][k]) + lds[3][k];
    if (t[0] > 0.0) write_record(A.mom, &q, 1, t, A.w, A.dt, A.tau_coef);
  }
}

AmrArgs amr_args(cc_ctx* ctx, const double* in, double* out) {
  AmrArgs A;
  A.in = in; A.out = out; A.G = ctx->a3;
  A.mom = ctx->s.mom; A.part = ctx->s.mpart;
  A.per_simple = ((ctx->a3.nsimple + 3) / 4 + 7) / 8;
  A.per = (ctx->a3.nreg - ctx->a3.nsimple + 7) / 8;      // one block per control volume
  A.per_irr = (ctx->a3.ncv - ctx->a3.nreg + 7) / 8;
  A.vmin = ctx->cfg.vmin; A.dv = ctx->dv; A.w = ctx->dv * ctx->dv * ctx->dv;
  A.dt = ctx->dt;
  A.tau_coef = ctx->cfg.kn > 0.0 ? sqrt(M_PI) / 2.0 * ctx->cfg.kn * ctx->cfg.lref / sqrt(2.0) : 0.0;
  A.t_wall = ctx->body.t_wall;
  A.om = ctx->body_state[5];
  A.cx = ctx->body.center[0]; A.cy = ctx->body.center[1];
  A.w0 = 0;
  return A;
}

typedef void (*amr_fn)(AmrArgs);

typedef void (*remap_fn)(const int*, const int*, const double*, const double*, double*, AmrArgs);

struct AmrFns { amr_fn simple, reg, irr, irr_mv, mom; remap_fn remap; };

template <int N>
AmrFns amr_fns() {
  return {k_amr_simple<N>, k_amr_step<N, false>, k_amr_step<N, true>, k_amr_step<N, true, true>, k_amr_mom<N>,
          k_amr_remap<N>};
}

bool pick_amr(int N, AmrFns* f) {
  switch (N) {
    case 4: *f = amr_fns<4>(); return true;
    case 6: *f = amr_fns<6>(); return true;
    case 8: *f = amr_fns<8>(); return true;
    case 12: *f = amr_fns<12>(); return true;
    case 16: *f = amr_fns<16>(); return true;
    default: return false;
  }
}

}  // namespace

hipError_t launch_amr_tables(cc_ctx* ctx) {
  const double* in = ctx->cfg.inflow;
  k_amr_tables<<<(ctx->nvel + 255) / 256, 256, 0, ctx->stream>>>(ctx->a3, ctx->N, ctx->cfg.vmin, ctx->dv, in[0],
                                                                  in[1], in[2], in[3], in[4]);
  return hipGetLastError();
}

hipError_t launch_amr_init(cc_ctx* ctx, const double* f) {
  const size_t tot = (size_t)ctx->ncell * ctx->nvel;
  k_amr_init<<<(unsigned)((tot + 255) / 256), 256, 0, ctx->stream>>>(ctx->a3, (double*)ctx->state[ctx->cur],
                                                                     ctx->nvel, f ? 1 : 0, f);
  return hipGetLastError();
}

hipError_t launch_amr_merge(cc_ctx* ctx, int from) {
  if (ctx->a3.ncv <= from) return hipSuccess;
  prof_begin(ctx, 3);
  k_amr_merge<<<ctx->a3.ncv - from, 256, 0, ctx->stream>>>(ctx->a3, (double*)ctx->state[ctx->cur], ctx->nvel, from);
  prof_end(ctx, 3);
  return hipGetLastError();
}

hipError_t launch_amr_moments(cc_ctx* ctx, int from) {
  AmrFns f;
  if (!pick_amr(ctx->N, &f)) return hipErrorNotSupported;
  if (ctx->a3.ncv <= from) return hipSuccess;
  const double* cur = (const double*)ctx->state[ctx->cur];
  AmrArgs A = amr_args(ctx, cur, nullptr);
  A.w0 = from;
  f.mom<<<(ctx->a3.ncv - from + 3) / 4, 256, 0, ctx->stream>>>(A);
  return hipGetLastError();
}

// one step state[cur] -> state[1-cur]; row (nullable) = force and mass of
// the state entering the step
hipError_t launch_amr_step(cc_ctx* ctx, double* row) {
  AmrFns f;
  if (!pick_amr(ctx->N, &f)) return hipErrorNotSupported;
  const double* in = (const double*)ctx->state[ctx->cur];
  double* out = (double*)ctx->state[1 - ctx->cur];
  const AmrArgs A = amr_args(ctx, in, out);
  // the few cut control volumes (too few waves to hide their latency on
  // their own) run on a side stream, overlapped with the streaming kernels
  const bool overlap = A.per_irr > 0 && ctx->side && !ctx->prof.on;
  hipError_t e = hipSuccess;
  if (overlap) {
    e = hipEventRecord(ctx->fork, ctx->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(ctx->side, ctx->fork, 0);
    if (e != hipSuccess) return e;
    (ctx->amr_turning ? f.irr_mv : f.irr)<<<A.per_irr * 8, 256, 0, ctx->side>>>(A);
    e = hipEventRecord(ctx->join, ctx->side);
    if (e != hipSuccess) return e;
  } else if (A.per_irr > 0) {
    prof_begin(ctx, 1);
    (ctx->amr_turning ? f.irr_mv : f.irr)<<<A.per_irr * 8, 256, 0, ctx->stream>>>(A);
    prof_end(ctx, 1);
  }
  prof_begin(ctx, 0);
  if (A.per_simple > 0) f.simple<<<A.per_simple * 8, 256, 0, ctx->stream>>>(A);
  if (A.per > 0) f.reg<<<A.per * 8, 256, 0, ctx->stream>>>(A);
  prof_end(ctx, 0);
  if (overlap) {
    e = hipStreamWaitEvent(ctx->stream, ctx->join, 0);
    if (e != hipSuccess) return e;
  }
  if (row) {
    prof_begin(ctx, 2);
    // blocks past the last control volume of each kind return at once and
    // write nothing: the partials are ceil(n_simple / 4) blocks of the
    // streaming kernel, then one per other control volume
    const int ns = ctx->a3.nsimple, nr = ctx->a3.nreg - ns, ni = ctx->a3.ncv - ctx->a3.nreg;
    k_amr_reduce<<<1, 1024, 0, ctx->stream>>>(ctx->s.mpart, (ns + 3) / 4 + nr + ni, row);
    prof_end(ctx, 2);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  ctx->cur = 1 - ctx->cur;
  ctx->nstep += 1;
  return hipSuccess;
}

hipError_t launch_amr_remap(cc_ctx* ctx, const double* from, double* to) {
  AmrFns f;
  if (!pick_amr(ctx->N, &f)) return hipErrorNotSupported;
  if (ctx->a3.nleaf == 0) return hipSuccess;
  prof_begin(ctx, 4);
  f.remap<<<ctx->a3.nleaf, 256, 0, ctx->stream>>>(ctx->a3.sptr, ctx->a3.src, ctx->a3.wgt, from, to,
                                                   amr_args(ctx, nullptr, nullptr));
  prof_end(ctx, 4);
  return hipGetLastError();
}

}  // namespace ccdvm
