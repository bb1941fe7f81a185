// Host side of the variable-degree entry points (dg_varp_* in dg.h): the
// elements of the (optionally refined) mesh, their node offsets, face table
// and per-(degree, size) element lists, the mortar tables, workspace
// carve-up and the launch sequence.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "dg_batch.h"
#include "dg_varp.h"

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// l^n_t(x) through the n points xi (product form).
double lagrange_at(const double* xi, int n, int t, double x) {
  double v = 1.0;
  for (int s = 0; s < n; ++s)
    if (s != t) v *= (x - xi[s]) / (xi[t] - xi[s]);
  return v;
}

struct Timed {
  hipEvent_t a, b;
  int slot;   // 3 p + mode, kMortarSlot or kHangSlot
};

constexpr int kMortarSlot = 3 * DG_VARP_MAXN;
constexpr int kHangSlot = kMortarSlot + 1;
// pencil of the element lists' visiting order (elements along x, planes
// along z), as the single-degree kernel's default
constexpr int kPencilX = 16;
constexpr int kPencilZ = 8;
constexpr int kSlots = kHangSlot + 1;

}  // namespace

struct dg_varp {
  int nx = 0, ny = 0, nz = 0;
  int64_t E = 0, T = 0;
  double gamma = 1.4;
  double L[3] = {1.0, 1.0, 1.0};
  int maxn = 0;
  std::vector<int> deg;          // per element
  std::vector<int> level;        // per element: 0 a whole cell, 1 a child of a refined cell
  std::vector<int64_t> off;      // E + 1
  std::vector<int> list;         // grouped by (degree, level)
  std::vector<int64_t> face;     // [E][6] (place << 2) | DG_FACE_*
  std::vector<DGVarpFace> faces; // mortar faces grouped by degree pair
  std::vector<DGVarpHang> hangs; // coarse faces with hanging faces, grouped by degree
  int64_t fbuf_doubles = 0;
  // ranges of the sorted mortar faces per degree pair (index lo * 9 + hi)
  // and of the sorted coarse faces per coarse point count
  int pair_first[(DG_VARP_MAXN + 1) * (DG_VARP_MAXN + 1)] = {};
  int pair_count[(DG_VARP_MAXN + 1) * (DG_VARP_MAXN + 1)] = {};
  int hang_first[DG_VARP_MAXN + 1] = {};
  int hang_count[DG_VARP_MAXN + 1] = {};
  // list range of point count N and level
  int first[DG_VARP_MAXN + 1][2] = {};
  int count[DG_VARP_MAXN + 1][2] = {};
  DGTables tab[DG_VARP_MAXN + 1][2];
  DGVarpTabs* htabs = nullptr;   // host copy
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool uploaded = false;
  bool timing = false;
  std::vector<Timed> ev;
  size_t ev_used = 0;
  ~dg_varp() {
    delete htabs;
    for (Timed& t : ev) {
      (void)hipEventDestroy(t.a);
      (void)hipEventDestroy(t.b);
    }
  }
};

namespace {

struct Layout {
  size_t off_tabs, off_off, off_face, off_list, off_faces, off_hangs, off_fbuf, off_tbuf, off_q2, total;
};

Layout layout(const dg_varp* v) {
  Layout L;
  L.off_tabs = 0;
  L.off_off = al256(sizeof(DGVarpTabs));
  L.off_face = L.off_off + al256(sizeof(int64_t) * (v->E + 1));
  L.off_list = L.off_face + al256(sizeof(int64_t) * 6 * v->E);
  L.off_faces = L.off_list + al256(sizeof(int) * v->E);
  L.off_hangs = L.off_faces + al256(sizeof(DGVarpFace) * v->faces.size());
  L.off_fbuf = L.off_hangs + al256(sizeof(DGVarpHang) * v->hangs.size());
  L.off_tbuf = L.off_fbuf + al256(sizeof(double) * v->fbuf_doubles);
  L.off_q2 = L.off_tbuf + al256(sizeof(double) * v->fbuf_doubles);
  L.total = L.off_q2 + al256((size_t)5 * v->T * sizeof(double));
  return L;
}

int hipfail(int err, const char* what) {
  return dg_set_error(DG_EHIP, "%s: HIP error %d (%s)", what, err, hipGetErrorString((hipError_t)err));
}

int ready(dg_varp* v) {
  if (!v) return dg_set_error(DG_EINVAL, "NULL variable-degree context");
  if (!v->ws) return dg_set_error(DG_EWORKSPACE, "no workspace set (need %zu bytes)", layout(v).total);
  if (!v->uploaded) return dg_set_error(DG_EWORKSPACE, "workspace not initialised (call dg_varp_set_workspace)");
  return DG_OK;
}

DGVarpMesh mesh_of(const dg_varp* v) {
  const Layout L = layout(v);
  DGVarpMesh m;
  m.tabs = (const DGVarpTabs*)(v->ws + L.off_tabs);
  m.off = (const int64_t*)(v->ws + L.off_off);
  m.face = (const int64_t*)(v->ws + L.off_face);
  m.list = (const int*)(v->ws + L.off_list);
  m.faces = (const DGVarpFace*)(v->ws + L.off_faces);
  m.hangs = (const DGVarpHang*)(v->ws + L.off_hangs);
  m.fbuf = (double*)(v->ws + L.off_fbuf);
  m.tbuf = (double*)(v->ws + L.off_tbuf);
  m.T = v->T;
  m.nfaces = (int)v->faces.size();
  m.nhangs = (int)v->hangs.size();
  return m;
}

int check_pair(const dg_varp* v, const void* a, const char* an, const void* b, const char* bn) {
  if (!a || !b) return dg_set_error(DG_EINVAL, "NULL %s", !a ? an : bn);
  if (((uintptr_t)a | (uintptr_t)b) & 7) return dg_set_error(DG_EINVAL, "arrays must be 8-byte aligned");
  const size_t sb = (size_t)5 * v->T * sizeof(double);
  if ((const char*)a < (const char*)b + sb && (const char*)b < (const char*)a + sb)
    return dg_set_error(DG_EALIAS, "%s overlaps %s", an, bn);
  return DG_OK;
}

// Event pair around a launch when timing is on (nullptr otherwise).
Timed* timer(dg_varp* v, int slot, int* err) {
  *err = 0;
  if (!v->timing || v->ev_used >= 65536) return nullptr;
  if (v->ev.size() <= v->ev_used) {
    Timed t;
    *err = (int)hipEventCreate(&t.a);
    if (*err) return nullptr;
    *err = (int)hipEventCreate(&t.b);
    if (*err) return nullptr;
    v->ev.push_back(t);
  }
  Timed* tm = &v->ev[v->ev_used++];
  tm->slot = slot;
  *err = (int)hipEventRecord(tm->a, v->stream);
  return tm;
}

// The mortar launches (one per degree pair present) and hanging-face
// launches (one per coarse degree present), each group timed as one, then
// one launch per (degree, level) present.  from_traces: the face launches
// read the traces that the stage launches producing Qin wrote; traces: the
// stage launches write those of Qout.
int launch_all(dg_varp* v, const double* Qin, double* Qout, double* RR, int mode, double a, double b, double dt,
               bool from_traces, bool traces) {
  const DGVarpMesh m = mesh_of(v);
  int err = 0;
  if (m.nfaces > 0) {
    Timed* tm = timer(v, kMortarSlot, &err);
    if (err) return err;
    for (int code = 0; code < (DG_VARP_MAXN + 1) * (DG_VARP_MAXN + 1); ++code) {
      if (!v->pair_count[code]) continue;
      err = dg_launch_varp_mortar(v->stream, v->tab[1][0], m, Qin, code / (DG_VARP_MAXN + 1),
                                  code % (DG_VARP_MAXN + 1), v->pair_first[code], v->pair_count[code], from_traces);
      if (err) return err;
    }
    if (tm && (err = (int)hipEventRecord(tm->b, v->stream))) return err;
  }
  if (m.nhangs > 0) {
    Timed* tm = timer(v, kHangSlot, &err);
    if (err) return err;
    for (int nc = 1; nc <= DG_VARP_MAXN; ++nc) {
      if (!v->hang_count[nc]) continue;
      err = dg_launch_varp_hanging(v->stream, v->tab[1][0], m, Qin, nc, v->hang_first[nc], v->hang_count[nc],
                                   from_traces);
      if (err) return err;
    }
    if (tm && (err = (int)hipEventRecord(tm->b, v->stream))) return err;
  }
  for (int N = v->maxn; N >= 1; --N) {
    for (int lev = 0; lev < 2; ++lev) {
      if (!v->count[N][lev]) continue;
      Timed* tm = timer(v, 3 * (N - 1) + mode, &err);
      if (err) return err;
      err = dg_launch_varp(v->stream, N, v->tab[N][lev], m, v->first[N][lev], v->count[N][lev], Qin, Qout, RR, mode,
                           a, b, dt, traces);
      if (err) return err;
      if (tm && (err = (int)hipEventRecord(tm->b, v->stream))) return err;
    }
  }
  return 0;
}

dg_varp* fail_null(int code, const char* what) {
  dg_set_error(code, "%s", what);
  return nullptr;
}

// The elements of the mesh (cell by cell; a refined cell's eight children in
// the order (kz, ky, kx), kx fastest), their offsets, face table, mortar and
// hanging faces, element lists and tables.  refine: NULL for no refinement.
dg_varp* build(int nx, int ny, int nz, const int* refine, const int* degrees, const double* L, double gamma) {
  if (nx < 1 || ny < 1 || nz < 1 || (int64_t)nx * ny * nz > 0x7fffffffLL) {
    dg_set_error(DG_EINVAL, "bad mesh size %d x %d x %d", nx, ny, nz);
    return nullptr;
  }
  if (!degrees || !L) return fail_null(DG_EINVAL, "NULL degrees or L");
  if (!(gamma > 1.0) || !std::isfinite(gamma)) return fail_null(DG_EINVAL, "gamma must be finite and > 1");
  if (!(L[0] > 0) || !(L[1] > 0) || !(L[2] > 0) || !std::isfinite(L[0] + L[1] + L[2]))
    return fail_null(DG_EINVAL, "domain lengths must be finite and > 0");
  const int64_t C = (int64_t)nx * ny * nz;
  int64_t E = 0;
  bool any_refined = false;
  for (int64_t c = 0; c < C; ++c) {
    const int r = refine ? refine[c] : 0;
    if (r != 0 && r != 1) {
      dg_set_error(DG_EINVAL, "cell %lld: refinement %d is not 0 or 1", (long long)c, r);
      return nullptr;
    }
    any_refined = any_refined || r;
    E += r ? 8 : 1;
  }
  if (E > 0x7fffffffLL || (any_refined && 8 * C > 0x7fffffffLL))
    return fail_null(DG_EUNSUPPORTED, "more than 2^31-1 elements");
  for (int64_t e = 0; e < E; ++e) {
    if (degrees[e] < 0 || degrees[e] >= DG_VARP_MAXN) {
      dg_set_error(DG_EUNSUPPORTED, "element %lld: degree %d outside 0..%d", (long long)e, degrees[e],
                   DG_VARP_MAXN - 1);
      return nullptr;
    }
  }
  dg_varp* v = new (std::nothrow) dg_varp;
  if (!v) return fail_null(DG_EINVAL, "out of host memory");
  v->htabs = new (std::nothrow) DGVarpTabs;
  if (!v->htabs) {
    delete v;
    return fail_null(DG_EINVAL, "out of host memory");
  }
  v->nx = nx;
  v->ny = ny;
  v->nz = nz;
  v->E = E;
  v->gamma = gamma;
  for (int d = 0; d < 3; ++d) v->L[d] = L[d];
  v->deg.assign(degrees, degrees + E);
  // elements cell by cell; cfirst[c]: the first element of cell c
  std::vector<int64_t> cfirst(C + 1);
  v->level.resize(E);
  {
    int64_t e = 0;
    for (int64_t c = 0; c < C; ++c) {
      cfirst[c] = e;
      const int n = (refine && refine[c]) ? 8 : 1;
      for (int k = 0; k < n; ++k) v->level[e++] = n == 8;
    }
    cfirst[C] = e;
  }
  v->off.resize(E + 1);
  int64_t T = 0;
  for (int64_t e = 0; e < E; ++e) {
    const int64_t n = v->deg[e] + 1;
    v->off[e] = T;
    T += n * n * n;
    v->maxn = std::max(v->maxn, (int)n);
  }
  v->off[E] = T;
  v->T = T;
  // element lists by (degree, level), each in the single-degree kernel's
  // visiting order over the cells: z-slabs of kPencilZ planes, inside a slab
  // pencils of kPencilX cells along x, inside a pencil y-row by y-row, then
  // z, x fastest; a refined cell's children together (an element's y- and
  // z-neighbours of the same group are listed close to it, so their reads
  // meet in L2)
  std::vector<int> cnt((DG_VARP_MAXN + 1) * 2, 0);
  for (int64_t e = 0; e < E; ++e) ++cnt[(v->deg[e] + 1) * 2 + v->level[e]];
  int pos = 0;
  for (int N = DG_VARP_MAXN; N >= 1; --N) {
    for (int lev = 0; lev < 2; ++lev) {
      v->first[N][lev] = pos;
      v->count[N][lev] = cnt[N * 2 + lev];
      pos += cnt[N * 2 + lev];
    }
  }
  v->list.resize(E);
  {
    std::vector<int> fill((DG_VARP_MAXN + 1) * 2, 0);
    for (int N = 1; N <= DG_VARP_MAXN; ++N)
      for (int lev = 0; lev < 2; ++lev) fill[N * 2 + lev] = v->first[N][lev];
    const int px = std::min(kPencilX, nx), pz = std::min(kPencilZ, nz);
    for (int zs = 0; zs < nz; zs += pz)
      for (int xs = 0; xs < nx; xs += px)
        for (int y = 0; y < ny; ++y)
          for (int z = zs; z < std::min(zs + pz, nz); ++z)
            for (int x = xs; x < std::min(xs + px, nx); ++x) {
              const int64_t c = ((int64_t)z * ny + y) * nx + x;
              for (int64_t e = cfirst[c]; e < cfirst[c + 1]; ++e)
                v->list[fill[(v->deg[e] + 1) * 2 + v->level[e]]++] = (int)e;
            }
  }
  // per-(degree, level) tables (the single-degree library's on the mesh of
  // that element size), Gauss-Legendre rules
  double xi[DG_VARP_MAXN + 1][DG_MAXN], w[DG_VARP_MAXN + 1][DG_MAXN];
  DGVarpTabs& H = *v->htabs;
  std::memset(&H, 0, sizeof(H));
  for (int N = 1; N <= DG_VARP_MAXN; ++N) {
    dg_build_tables(nx, ny, nz, N - 1, gamma, v->L, &v->tab[N][0], xi[N], w[N]);
    if (any_refined)
      dg_build_tables(2 * nx, 2 * ny, 2 * nz, N - 1, gamma, v->L, &v->tab[N][1], xi[N], w[N]);
    else
      v->tab[N][1] = v->tab[N][0];
    for (int m = 0; m < N; ++m) {
      H.lm[N][m] = v->tab[N][0].lm[m];
      H.lp[N][m] = v->tab[N][0].lp[m];
    }
  }
  for (int n = 1; n <= DG_VARP_MAXN; ++n) {
    for (int M = n; M <= DG_VARP_MAXN; ++M) {
      for (int b = 0; b < M; ++b) {
        for (int t = 0; t < n; ++t) {
          if (M > n) {
            const double l = lagrange_at(xi[n], n, t, xi[M][b]);
            H.interp[n][M][b * n + t] = l;
            H.proj[n][M][t * M + b] = l * w[M][b] / w[n][t];
          }
          for (int h = 0; h < 2; ++h) {
            const double l = lagrange_at(xi[n], n, t, 0.5 * (xi[M][b] + 2 * h - 1));
            H.hinterp[n][M][h][b * n + t] = l;
            H.hproj[n][M][h][t * M + b] = 0.5 * l * w[M][b] / w[n][t];
          }
        }
      }
    }
  }
  // faces: every element's +d face once, as the oracle's enumeration: a
  // sibling or a same-size neighbour (conforming, or a mortar face between
  // degrees), or hanging sub-faces (fine against coarse: one; coarse
  // against a refined cell: four)
  v->face.assign(6 * E, -1);
  auto el_of = [&](int64_t c, int kx, int ky, int kz) { return cfirst[c] + (kz * 2 + ky) * 2 + kx; };
  auto same_size = [&](int64_t a, int64_t b, int d) {
    const int na = v->deg[a] + 1, nb = v->deg[b] + 1;
    if (na == nb) {
      v->face[6 * a + 2 * d + 1] = (v->off[b] << 2) | DG_FACE_CONFORMING;
      v->face[6 * b + 2 * d] = (v->off[a] << 2) | DG_FACE_CONFORMING;
      return;
    }
    DGVarpFace F;
    F.oa = v->off[a];
    F.ob = v->off[b];
    F.d = d;
    const int lo = std::min(na, nb), hi = std::max(na, nb);
    F.code = (lo * (DG_VARP_MAXN + 1) + hi) * 2 + (na < nb ? 1 : 0);
    F.sa = v->fbuf_doubles;
    v->fbuf_doubles += 5 * (int64_t)na * na;
    F.sb = v->fbuf_doubles;
    v->fbuf_doubles += 5 * (int64_t)nb * nb;
    v->face[6 * a + 2 * d + 1] = (F.sa << 2) | DG_FACE_MORTAR;
    v->face[6 * b + 2 * d] = (F.sb << 2) | DG_FACE_MORTAR;
    v->faces.push_back(F);
  };
  // quarter (q1, q2) of coarse element ec's face 2d + cside against fine
  // element ef: the coarse face's record (its summed projection block) on
  // first use, the fine side's block per quarter
  std::vector<int64_t> hang_of(any_refined ? 6 * E : 0, -1);
  auto hanging = [&](int64_t ec, int64_t ef, int d, int cside, int q1, int q2) {
    const int nc = v->deg[ec] + 1, nf = v->deg[ef] + 1;
    int64_t& hi = hang_of[6 * ec + 2 * d + cside];
    if (hi < 0) {
      DGVarpHang G{};
      G.oc = v->off[ec];
      G.sc = v->fbuf_doubles;
      v->fbuf_doubles += 5 * (int64_t)nc * nc;
      G.d = d;
      G.nc = nc;
      G.cminus = cside;
      for (int q = 0; q < 4; ++q) G.nf[q] = 0;
      v->face[6 * ec + 2 * d + cside] = (G.sc << 2) | DG_FACE_MORTAR;
      hi = (int64_t)v->hangs.size();
      v->hangs.push_back(G);
    }
    DGVarpHang& G = v->hangs[hi];
    const int q = 2 * q2 + q1;
    G.of[q] = v->off[ef];
    G.sf[q] = v->fbuf_doubles;
    G.nf[q] = nf;
    v->fbuf_doubles += 5 * (int64_t)nf * nf;
    v->face[6 * ef + 2 * d + (1 - cside)] = (G.sf[q] << 2) | DG_FACE_MORTAR;
  };
  for (int64_t c = 0; c < C; ++c) {
    const int cx = (int)(c % nx), cy = (int)((c / nx) % ny), cz = (int)(c / ((int64_t)nx * ny));
    const bool rc = refine && refine[c];
    for (int d = 0; d < 3; ++d) {
      const int x = d == 0 ? (cx + 1) % nx : cx, y = d == 1 ? (cy + 1) % ny : cy, z = d == 2 ? (cz + 1) % nz : cz;
      const int64_t cn = ((int64_t)z * ny + y) * nx + x;
      const bool rn = refine && refine[cn];
      const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;   // tangential axes, ascending
      if (!rc && !rn) {
        same_size(cfirst[c], cfirst[cn], d);
        continue;
      }
      for (int kz = 0; kz < 2; ++kz)
        for (int ky = 0; ky < 2; ++ky)
          for (int kx = 0; kx < 2; ++kx) {
            int k[3] = {kx, ky, kz};
            if (rc) {
              const int64_t e = el_of(c, kx, ky, kz);
              if (k[d] == 0) {   // the sibling across the cell's midplane
                k[d] = 1;
                same_size(e, el_of(c, k[0], k[1], k[2]), d);
              } else if (rn) {   // the neighbour cell's child across the cell face
                k[d] = 0;
                same_size(e, el_of(cn, k[0], k[1], k[2]), d);
              } else {           // fine e (-d side) against the coarse neighbour
                hanging(cfirst[cn], e, d, 0, k[t0], k[t1]);
              }
            } else if (k[d] == 0) {   // coarse c (-d side) against the refined neighbour's children
              hanging(cfirst[c], el_of(cn, kx, ky, kz), d, 1, k[t0], k[t1]);
            }
          }
    }
  }
  for (int64_t i = 0; i < 6 * E; ++i) {
    if (v->face[i] < 0) {
      delete v;
      return fail_null(DG_EINVAL, "internal error: an element face without a neighbour");
    }
  }
  if (v->faces.size() > 0x7fffffffu || v->hangs.size() > 0x7fffffffu) {
    delete v;
    return fail_null(DG_EUNSUPPORTED, "more than 2^31-1 faces between degrees or coarse faces with hanging faces");
  }
  // waves that run together mostly take the same kernel branch
  std::stable_sort(v->faces.begin(), v->faces.end(),
                   [](const DGVarpFace& a, const DGVarpFace& b) { return (a.code >> 1) < (b.code >> 1); });
  for (const DGVarpHang& G : v->hangs) {
    if (!G.nf[0] || !G.nf[1] || !G.nf[2] || !G.nf[3]) {
      delete v;
      return fail_null(DG_EINVAL, "internal error: a coarse face without its four quarters");
    }
  }
  std::stable_sort(v->hangs.begin(), v->hangs.end(),
                   [](const DGVarpHang& a, const DGVarpHang& b) { return a.nc < b.nc; });
  for (size_t i = 0; i < v->faces.size(); ++i) {
    const int code = v->faces[i].code >> 1;
    if (!v->pair_count[code]) v->pair_first[code] = (int)i;
    ++v->pair_count[code];
  }
  for (size_t i = 0; i < v->hangs.size(); ++i) {
    const int nc = v->hangs[i].nc;
    if (!v->hang_count[nc]) v->hang_first[nc] = (int)i;
    ++v->hang_count[nc];
  }
  dg_set_error(DG_OK, "");
  return v;
}

}  // namespace

extern "C" {

dg_varp* dg_varp_create(int nx, int ny, int nz, const int* degrees, const double* L, double gamma) {
  return build(nx, ny, nz, nullptr, degrees, L, gamma);
}

dg_varp* dg_varp_create_refined(int nx, int ny, int nz, const int* refine, const int* degrees, const double* L,
                                double gamma) {
  if (!refine) return fail_null(DG_EINVAL, "NULL refine");
  return build(nx, ny, nz, refine, degrees, L, gamma);
}

void dg_varp_destroy(dg_varp* v) { delete v; }

int dg_varp_set_stream(dg_varp* v, void* s) {
  if (!v) return dg_set_error(DG_EINVAL, "NULL variable-degree context");
  v->stream = (hipStream_t)s;
  return DG_OK;
}

int64_t dg_varp_num_dof(const dg_varp* v) { return v ? v->T : -1; }

int64_t dg_varp_num_elements(const dg_varp* v) { return v ? v->E : -1; }

int64_t dg_varp_offset(const dg_varp* v, int64_t e) {
  if (!v || e < 0 || e > v->E) return -1;
  return v->off[e];
}

size_t dg_varp_workspace_bytes(const dg_varp* v) { return v ? layout(v).total : 0; }

int dg_varp_set_workspace(dg_varp* v, void* dptr, size_t bytes) {
  if (!v) return dg_set_error(DG_EINVAL, "NULL variable-degree context");
  if (!dptr) return dg_set_error(DG_EINVAL, "NULL workspace");
  if (((uintptr_t)dptr) & 255) return dg_set_error(DG_EINVAL, "workspace not 256-byte aligned");
  const Layout L = layout(v);
  if (bytes < L.total) return dg_set_error(DG_EWORKSPACE, "workspace %zu bytes < %zu", bytes, L.total);
  v->ws = (char*)dptr;
  v->ws_bytes = bytes;
  v->uploaded = false;
  int err = (int)hipMemcpy(v->ws + L.off_tabs, v->htabs, sizeof(DGVarpTabs), hipMemcpyHostToDevice);
  if (err) return hipfail(err, "upload mortar tables");
  err = (int)hipMemcpy(v->ws + L.off_face, v->face.data(), sizeof(int64_t) * 6 * v->E, hipMemcpyHostToDevice);
  if (err) return hipfail(err, "upload face table");
  if (!v->faces.empty()) {
    err = (int)hipMemcpy(v->ws + L.off_faces, v->faces.data(), sizeof(DGVarpFace) * v->faces.size(),
                         hipMemcpyHostToDevice);
    if (err) return hipfail(err, "upload mortar faces");
  }
  if (!v->hangs.empty()) {
    err = (int)hipMemcpy(v->ws + L.off_hangs, v->hangs.data(), sizeof(DGVarpHang) * v->hangs.size(),
                         hipMemcpyHostToDevice);
    if (err) return hipfail(err, "upload hanging faces");
  }
  err = (int)hipMemcpy(v->ws + L.off_off, v->off.data(), sizeof(int64_t) * (v->E + 1), hipMemcpyHostToDevice);
  if (err) return hipfail(err, "upload offsets");
  err = (int)hipMemcpy(v->ws + L.off_list, v->list.data(), sizeof(int) * v->E, hipMemcpyHostToDevice);
  if (err) return hipfail(err, "upload element lists");
  v->uploaded = true;
  return DG_OK;
}

int dg_varp_rhs(dg_varp* v, const double* Q, double* R) {
  int rc = ready(v);
  if (rc) return rc;
  rc = check_pair(v, Q, "Q", R, "R");
  if (rc) return rc;
  const int err = launch_all(v, Q, nullptr, R, 0, 0.0, 0.0, 0.0, false, false);
  if (err) return hipfail(err, "variable-degree rhs launch");
  return DG_OK;
}

int dg_varp_rk_steps(dg_varp* v, double* Q, double* res, double dt, int nsteps) {
  int rc = ready(v);
  if (rc) return rc;
  rc = check_pair(v, Q, "Q", res, "res");
  if (rc) return rc;
  if (nsteps < 0) return dg_set_error(DG_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(dt)) return dg_set_error(DG_EINVAL, "dt not finite");
  double* buf[2] = {Q, (double*)(v->ws + layout(v).off_q2)};
  // the first stage's face launches form the traces of Q from its state;
  // every stage launch writes the traces of its output for the next stage
  const bool faces = !v->faces.empty() || !v->hangs.empty();
  for (int n = 0; n < nsteps; ++n) {
    for (int s = 0; s < 5; ++s) {
      const int g = (n & 1) + s;
      const bool first = n == 0 && s == 0, last = n == nsteps - 1 && s == 4;
      const int err = launch_all(v, buf[g & 1], buf[(g + 1) & 1], res, s == 0 ? 2 : 1, kDgRKA[s], kDgRKB[s], dt,
                                 faces && !first, faces && !last);
      if (err) return hipfail(err, "variable-degree stage launch");
    }
  }
  if (nsteps & 1) {
    const int err =
        (int)hipMemcpyAsync(Q, buf[1], (size_t)5 * v->T * sizeof(double), hipMemcpyDeviceToDevice, v->stream);
    if (err) return hipfail(err, "state copy");
  }
  return DG_OK;
}

int dg_varp_set_timing(dg_varp* v, int on) {
  if (!v) return dg_set_error(DG_EINVAL, "NULL variable-degree context");
  v->timing = on != 0;
  v->ev_used = 0;
  return DG_OK;
}

int dg_varp_timing_read(dg_varp* v, double* ms, int64_t* count) {
  if (!v || !ms || !count) return dg_set_error(DG_EINVAL, "NULL argument");
  for (int i = 0; i < kSlots; ++i) {
    ms[i] = 0.0;
    count[i] = 0;
  }
  for (size_t i = 0; i < v->ev_used; ++i) {
    const Timed& t = v->ev[i];
    int err = (int)hipEventSynchronize(t.b);
    if (err) return hipfail(err, "timing event");
    float x = 0.f;
    err = (int)hipEventElapsedTime(&x, t.a, t.b);
    if (err) return hipfail(err, "timing read");
    ms[t.slot] += x;
    count[t.slot] += 1;
  }
  v->ev_used = 0;
  return DG_OK;
}

}  // extern "C"
