// Host side of the variable-degree entry points (dg_varp_* in dg.h): the
// per-degree element lists, node offsets, mortar tables, workspace carve-up
// and the per-degree launch sequence.

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
  int slot;   // 3 p + mode, or kMortarSlot
};

constexpr int kMortarSlot = 3 * DG_VARP_MAXN;
// pencil of the element lists' visiting order (elements along x, planes
// along z), as the single-degree kernel's default
constexpr int kPencilX = 16;
constexpr int kPencilZ = 8;
constexpr int kSlots = kMortarSlot + 1;

}  // namespace

struct dg_varp {
  int nx = 0, ny = 0, nz = 0;
  int64_t E = 0, T = 0;
  double gamma = 1.4;
  double L[3] = {1.0, 1.0, 1.0};
  int maxn = 0;
  std::vector<int> deg;          // per element
  std::vector<int64_t> off;      // E + 1
  std::vector<int> list;         // grouped by degree
  std::vector<int64_t> slot;     // [E][6] mortar flux place, -1 where conforming
  std::vector<DGVarpFace> faces; // mortar faces grouped by degree pair
  int64_t fbuf_doubles = 0;
  int first[DG_VARP_MAXN + 1] = {0};   // list range of point count N
  int count[DG_VARP_MAXN + 1] = {0};
  DGTables tab[DG_VARP_MAXN + 1];
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
  size_t off_tabs, off_off, off_slot, off_list, off_faces, off_fbuf, off_q2, total;
};

Layout layout(const dg_varp* v) {
  Layout L;
  L.off_tabs = 0;
  L.off_off = al256(sizeof(DGVarpTabs));
  L.off_slot = L.off_off + al256(sizeof(int64_t) * (v->E + 1));
  L.off_list = L.off_slot + al256(sizeof(int64_t) * 6 * v->E);
  L.off_faces = L.off_list + al256(sizeof(int) * v->E);
  L.off_fbuf = L.off_faces + al256(sizeof(DGVarpFace) * v->faces.size());
  L.off_q2 = L.off_fbuf + al256(sizeof(double) * v->fbuf_doubles);
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
  m.slot = (const int64_t*)(v->ws + L.off_slot);
  m.list = (const int*)(v->ws + L.off_list);
  m.faces = (const DGVarpFace*)(v->ws + L.off_faces);
  m.fbuf = (double*)(v->ws + L.off_fbuf);
  m.T = v->T;
  m.nx = v->nx;
  m.ny = v->ny;
  m.nz = v->nz;
  m.nfaces = (int)v->faces.size();
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

// The mortar launch, then one launch per degree present.
int launch_all(dg_varp* v, const double* Qin, double* Qout, double* RR, int mode, double a, double b, double dt) {
  const DGVarpMesh m = mesh_of(v);
  int err = 0;
  if (m.nfaces > 0) {
    Timed* tm = timer(v, kMortarSlot, &err);
    if (err) return err;
    err = dg_launch_varp_mortar(v->stream, v->tab[1], m, Qin);
    if (err) return err;
    if (tm && (err = (int)hipEventRecord(tm->b, v->stream))) return err;
  }
  for (int N = v->maxn; N >= 1; --N) {
    if (!v->count[N]) continue;
    Timed* tm = timer(v, 3 * (N - 1) + mode, &err);
    if (err) return err;
    err = dg_launch_varp(v->stream, N, v->tab[N], m, v->first[N], v->count[N], Qin, Qout, RR, mode, a, b, dt);
    if (err) return err;
    if (tm && (err = (int)hipEventRecord(tm->b, v->stream))) return err;
  }
  return 0;
}

}  // namespace

extern "C" {

dg_varp* dg_varp_create(int nx, int ny, int nz, const int* degrees, const double* L, double gamma) {
  if (nx < 1 || ny < 1 || nz < 1 || (int64_t)nx * ny * nz > 0x7fffffffLL) {
    dg_set_error(DG_EINVAL, "bad mesh size %d x %d x %d", nx, ny, nz);
    return nullptr;
  }
  if (!degrees || !L) {
    dg_set_error(DG_EINVAL, "NULL degrees or L");
    return nullptr;
  }
  if (!(gamma > 1.0) || !std::isfinite(gamma)) {
    dg_set_error(DG_EINVAL, "gamma must be finite and > 1");
    return nullptr;
  }
  if (!(L[0] > 0) || !(L[1] > 0) || !(L[2] > 0) || !std::isfinite(L[0] + L[1] + L[2])) {
    dg_set_error(DG_EINVAL, "domain lengths must be finite and > 0");
    return nullptr;
  }
  const int64_t E = (int64_t)nx * ny * nz;
  for (int64_t e = 0; e < E; ++e) {
    if (degrees[e] < 0 || degrees[e] >= DG_VARP_MAXN) {
      dg_set_error(DG_EUNSUPPORTED, "element %lld: degree %d outside 0..%d", (long long)e, degrees[e],
                   DG_VARP_MAXN - 1);
      return nullptr;
    }
  }
  dg_varp* v = new (std::nothrow) dg_varp;
  if (!v) {
    dg_set_error(DG_EINVAL, "out of host memory");
    return nullptr;
  }
  v->htabs = new (std::nothrow) DGVarpTabs;
  if (!v->htabs) {
    delete v;
    dg_set_error(DG_EINVAL, "out of host memory");
    return nullptr;
  }
  v->nx = nx;
  v->ny = ny;
  v->nz = nz;
  v->E = E;
  v->gamma = gamma;
  for (int d = 0; d < 3; ++d) v->L[d] = L[d];
  v->deg.assign(degrees, degrees + E);
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
  // element lists by degree, each in the single-degree kernel's visiting
  // order: z-slabs of kPencilZ planes, inside a slab pencils of kPencilX
  // elements along x, inside a pencil y-row by y-row, then z, x fastest (an
  // element's y- and z-neighbours of the same degree are listed close to
  // it, so their reads meet in L2)
  std::vector<int> cnt(DG_VARP_MAXN + 1, 0);
  for (int64_t e = 0; e < E; ++e) ++cnt[v->deg[e] + 1];
  int pos = 0;
  for (int N = DG_VARP_MAXN; N >= 1; --N) {
    v->first[N] = pos;
    v->count[N] = cnt[N];
    pos += cnt[N];
  }
  v->list.resize(E);
  std::vector<int> fill(v->first, v->first + DG_VARP_MAXN + 1);
  {
    const int px = std::min(kPencilX, nx), pz = std::min(kPencilZ, nz);
    for (int zs = 0; zs < nz; zs += pz)
      for (int xs = 0; xs < nx; xs += px)
        for (int y = 0; y < ny; ++y)
          for (int z = zs; z < std::min(zs + pz, nz); ++z)
            for (int x = xs; x < std::min(xs + px, nx); ++x) {
              const int64_t e = ((int64_t)z * ny + y) * nx + x;
              v->list[fill[v->deg[e] + 1]++] = (int)e;
            }
  }
  // per-degree tables (the single-degree library's), Gauss-Legendre rules
  double xi[DG_VARP_MAXN + 1][DG_MAXN], w[DG_VARP_MAXN + 1][DG_MAXN];
  DGVarpTabs& H = *v->htabs;
  std::memset(&H, 0, sizeof(H));
  for (int N = 1; N <= DG_VARP_MAXN; ++N) {
    dg_build_tables(nx, ny, nz, N - 1, gamma, v->L, &v->tab[N], xi[N], w[N]);
    for (int m = 0; m < N; ++m) {
      H.lm[N][m] = v->tab[N].lm[m];
      H.lp[N][m] = v->tab[N].lp[m];
    }
  }
  for (int n = 1; n <= DG_VARP_MAXN; ++n) {
    for (int M = n + 1; M <= DG_VARP_MAXN; ++M) {
      for (int b = 0; b < M; ++b) {
        for (int t = 0; t < n; ++t) {
          const double l = lagrange_at(xi[n], n, t, xi[M][b]);
          H.interp[n][M][b * n + t] = l;
          H.proj[n][M][t * M + b] = l * w[M][b] / w[n][t];
        }
      }
    }
  }
  // mortar faces: every +d face whose neighbour has another degree; each
  // side's projected flux gets its own place in the face-flux buffer
  v->slot.assign(6 * E, -1);
  for (int64_t e = 0; e < E; ++e) {
    const int ex = (int)(e % nx), ey = (int)((e / nx) % ny), ez = (int)(e / ((int64_t)nx * ny));
    for (int d = 0; d < 3; ++d) {
      const int x = d == 0 ? (ex + 1) % nx : ex, y = d == 1 ? (ey + 1) % ny : ey, z = d == 2 ? (ez + 1) % nz : ez;
      const int64_t nb = ((int64_t)z * ny + y) * nx + x;
      const int na = v->deg[e] + 1, nn = v->deg[nb] + 1;
      if (na == nn) continue;
      DGVarpFace F;
      F.oa = v->off[e];
      F.ob = v->off[nb];
      F.d = d;
      const int lo = std::min(na, nn), hi = std::max(na, nn);
      F.code = (lo * (DG_VARP_MAXN + 1) + hi) * 2 + (na < nn ? 1 : 0);
      F.sa = v->fbuf_doubles;
      v->fbuf_doubles += 5 * (int64_t)na * na;
      F.sb = v->fbuf_doubles;
      v->fbuf_doubles += 5 * (int64_t)nn * nn;
      v->slot[6 * e + 2 * d + 1] = F.sa;
      v->slot[6 * nb + 2 * d] = F.sb;
      v->faces.push_back(F);
    }
  }
  if (v->faces.size() > 0x7fffffffu) {
    delete v;
    dg_set_error(DG_EUNSUPPORTED, "more than 2^31-1 faces between degrees");
    return nullptr;
  }
  // waves that run together mostly take the same degree pair
  std::stable_sort(v->faces.begin(), v->faces.end(),
                   [](const DGVarpFace& x, const DGVarpFace& y) { return (x.code >> 1) < (y.code >> 1); });
  dg_set_error(DG_OK, "");
  return v;
}

void dg_varp_destroy(dg_varp* v) { delete v; }

int dg_varp_set_stream(dg_varp* v, void* s) {
  if (!v) return dg_set_error(DG_EINVAL, "NULL variable-degree context");
  v->stream = (hipStream_t)s;
  return DG_OK;
}

int64_t dg_varp_num_dof(const dg_varp* v) { return v ? v->T : -1; }

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
  err = (int)hipMemcpy(v->ws + L.off_slot, v->slot.data(), sizeof(int64_t) * 6 * v->E, hipMemcpyHostToDevice);
  if (err) return hipfail(err, "upload face slots");
  if (!v->faces.empty()) {
    err = (int)hipMemcpy(v->ws + L.off_faces, v->faces.data(), sizeof(DGVarpFace) * v->faces.size(),
                         hipMemcpyHostToDevice);
    if (err) return hipfail(err, "upload mortar faces");
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
  const int err = launch_all(v, Q, nullptr, R, 0, 0.0, 0.0, 0.0);
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
  for (int n = 0; n < nsteps; ++n) {
    for (int s = 0; s < 5; ++s) {
      const int g = (n & 1) + s;
      const int err = launch_all(v, buf[g & 1], buf[(g + 1) & 1], res, s == 0 ? 2 : 1, kDgRKA[s], kDgRKB[s], dt);
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
