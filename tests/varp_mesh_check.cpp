// Host check of the variable-degree builder (the mesh, face table, mortar and
// hanging faces, element lists and face-flux buffer that dg_varp_create and
// dg_varp_create_refined set up), compiled with the builder's own source
// and linked against the library for the table and kernel-launch symbols
// (nothing here touches a GPU).  For seeded random refinements and degrees
// on meshes one to five cells across:
//   - every element face names a place of its kind: a conforming neighbour
//     is the element that touches that face geometrically and has the same
//     size and degree; a mortar or hanging face points into the face-flux
//     buffer;
//   - every mortar face joins two touching elements of the same size and
//     different degrees, with the degree pair its code names;
//   - every coarse face with hanging faces has one record, whose quarter
//     q = 2 q2 + q1 is the whole face of a fine element touching across it;
//   - the kernels write every double of the face-flux buffer exactly once,
//     and every element face reads only written doubles of its own blocks;
//   - the element lists hold every element once, grouped by (degree, size),
//     and the launch ranges of the mortar and hanging faces every face once.
// Exit status 0 and "ok" on success.
#include "varp_api.cpp"

#include <cstdio>
#include <random>

namespace {

int fails = 0;

#define CHECK(cond, ...)          \
  do {                            \
    if (!(cond)) {                \
      if (fails++ < 20) {         \
        printf(__VA_ARGS__);      \
        printf("\n");             \
      }                           \
    }                             \
  } while (0)

// Element geometry in units of half a cell: origin and size per direction.
struct Geo {
  int x0[3], s;
};

int check_mesh(int nx, int ny, int nz, const std::vector<int>& ref, std::mt19937& rng) {
  const int n[3] = {nx, ny, nz};
  std::vector<Geo> geo;
  for (int cz = 0; cz < nz; ++cz)
    for (int cy = 0; cy < ny; ++cy)
      for (int cx = 0; cx < nx; ++cx) {
        const int c = (cz * ny + cy) * nx + cx;
        if (ref[c]) {
          for (int k = 0; k < 8; ++k) geo.push_back({{2 * cx + (k & 1), 2 * cy + ((k >> 1) & 1), 2 * cz + (k >> 2)}, 1});
        } else {
          geo.push_back({{2 * cx, 2 * cy, 2 * cz}, 2});
        }
      }
  const int64_t E = (int64_t)geo.size();
  std::vector<int> deg(E);
  std::uniform_int_distribution<int> pd(0, 7);
  const int pmax = pd(rng);
  for (int64_t e = 0; e < E; ++e) deg[e] = std::uniform_int_distribution<int>(0, pmax)(rng);
  const double L[3] = {1.0, 0.8, 1.2};
  dg_varp* v = dg_varp_create_refined(nx, ny, nz, ref.data(), deg.data(), L, 1.4);
  if (!v) {
    printf("create failed: %s\n", dg_last_error());
    return 1;
  }
  CHECK(v->E == E, "element count %lld != %lld", (long long)v->E, (long long)E);
  std::vector<int64_t> elem_at;   // first node -> element
  std::vector<int64_t> first_of(E);
  for (int64_t e = 0; e < E; ++e) first_of[e] = v->off[e];
  auto element_at = [&](int64_t node) -> int64_t {
    auto it = std::lower_bound(first_of.begin(), first_of.end(), node);
    if (it == first_of.end() || *it != node) return -1;
    return it - first_of.begin();
  };
  // does b touch a's +d face (b on the +d side), covering exactly the same
  // rectangle (same size) -- periodic in units of half a cell
  auto wrap = [&](int x, int d) { return ((x % (2 * n[d])) + 2 * n[d]) % (2 * n[d]); };
  auto touches_plus = [&](int64_t a, int64_t b, int d) {
    const Geo &A = geo[a], &B = geo[b];
    if (wrap(A.x0[d] + A.s, d) != wrap(B.x0[d], d)) return false;
    for (int t = 0; t < 3; ++t)
      if (t != d && A.x0[t] != B.x0[t]) return false;
    return A.s == B.s;
  };
  const int64_t nb = v->fbuf_doubles;
  std::vector<int> written(nb, 0);
  auto write = [&](int64_t s, int64_t len, const char* what) {
    CHECK(s >= 0 && s + len <= nb, "%s block [%lld, %lld) outside the buffer of %lld", what, (long long)s,
          (long long)(s + len), (long long)nb);
    if (s < 0 || s + len > nb) return;
    for (int64_t i = s; i < s + len; ++i) ++written[i];
  };
  for (const DGVarpFace& F : v->faces) {
    const int64_t a = element_at(F.oa), b = element_at(F.ob);
    CHECK(a >= 0 && b >= 0, "mortar face names no element");
    if (a < 0 || b < 0) continue;
    CHECK(touches_plus(a, b, F.d), "mortar face %lld -> %lld along %d does not touch", (long long)a, (long long)b,
          F.d);
    const int na = deg[a] + 1, nb2 = deg[b] + 1;
    CHECK(na != nb2, "mortar face between equal degrees");
    const int lo = std::min(na, nb2), hi = std::max(na, nb2);
    CHECK(F.code == (lo * (DG_VARP_MAXN + 1) + hi) * 2 + (na < nb2 ? 1 : 0), "mortar code");
    write(F.sa, 5LL * na * na, "mortar a");
    write(F.sb, 5LL * nb2 * nb2, "mortar b");
  }
  std::vector<int> coarse_seen(6 * E, 0);
  for (const DGVarpHang& H : v->hangs) {
    const int64_t c = element_at(H.oc);
    CHECK(c >= 0, "hanging face names no coarse element");
    if (c < 0) continue;
    const int d = H.d, t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
    CHECK(d >= 0 && d < 3 && geo[c].s == 2 && H.nc == deg[c] + 1, "coarse side of a hanging face");
    const int cface = 2 * d + (H.cminus ? 1 : 0);
    CHECK(++coarse_seen[6 * c + cface] == 1, "coarse face %lld/%d has two records", (long long)c, cface);
    CHECK(v->face[6 * c + cface] == ((H.sc << 2) | DG_FACE_MORTAR), "coarse face does not name its block");
    write(H.sc, 5LL * H.nc * H.nc, "hanging coarse");
    const Geo& C = geo[c];
    for (int q = 0; q < 4; ++q) {
      const int64_t f = element_at(H.of[q]);
      CHECK(f >= 0, "hanging face names no fine element");
      if (f < 0) continue;
      const Geo& Fi = geo[f];
      CHECK(Fi.s == 1 && H.nf[q] == deg[f] + 1, "fine side of quarter %d", q);
      if (H.cminus) {
        CHECK(wrap(C.x0[d] + 2, d) == wrap(Fi.x0[d], d), "coarse -d side does not touch");
      } else {
        CHECK(wrap(Fi.x0[d] + 1, d) == wrap(C.x0[d], d), "fine -d side does not touch");
      }
      CHECK(Fi.x0[t0] == C.x0[t0] + (q & 1) && Fi.x0[t1] == C.x0[t1] + (q >> 1), "fine face is not quarter %d", q);
      const int64_t ff = v->face[6 * f + 2 * d + (H.cminus ? 0 : 1)];
      CHECK(ff == ((H.sf[q] << 2) | DG_FACE_MORTAR), "fine face of a hanging face does not name its block");
      write(H.sf[q], 5LL * H.nf[q] * H.nf[q], "hanging fine");
    }
  }
  for (int64_t i = 0; i < nb; ++i) CHECK(written[i] == 1, "buffer double %lld written %d times", (long long)i,
                                         written[i]);
  for (int64_t e = 0; e < E; ++e) {
    const int N = deg[e] + 1;
    for (int f = 0; f < 6; ++f) {
      const int64_t fr = v->face[6 * e + f];
      const int kind = (int)(fr & 3), d = f >> 1, side = f & 1;
      const int64_t place = fr >> 2;
      CHECK(fr >= 0 && kind <= DG_FACE_MORTAR, "element %lld face %d unset", (long long)e, f);
      if (kind == DG_FACE_CONFORMING) {
        const int64_t b = element_at(place);
        CHECK(b >= 0, "conforming face names no element");
        if (b < 0) continue;
        CHECK(deg[b] == deg[e], "conforming face between degrees");
        CHECK(side ? touches_plus(e, b, d) : touches_plus(b, e, d), "conforming neighbour of %lld face %d is wrong",
              (long long)e, f);
      } else {
        const int64_t len = 5LL * N * N;
        CHECK(place >= 0 && place + len <= nb, "face block outside the buffer");
        if (place < 0 || place + len > nb) continue;
        for (int64_t i = place; i < place + len; ++i) CHECK(written[i] == 1, "face reads an unwritten double");
      }
    }
  }
  // the per-launch ranges: each degree pair's mortar faces and each coarse
  // degree's coarse faces, together every face once
  int64_t nface = 0, nhang = 0;
  for (int code = 0; code < (DG_VARP_MAXN + 1) * (DG_VARP_MAXN + 1); ++code) {
    for (int i = v->pair_first[code]; i < v->pair_first[code] + v->pair_count[code]; ++i)
      CHECK(i >= 0 && i < (int)v->faces.size() && (v->faces[i].code >> 1) == code, "mortar range of pair %d", code);
    nface += v->pair_count[code];
  }
  for (int nc = 0; nc <= DG_VARP_MAXN; ++nc) {
    for (int i = v->hang_first[nc]; i < v->hang_first[nc] + v->hang_count[nc]; ++i)
      CHECK(i >= 0 && i < (int)v->hangs.size() && v->hangs[i].nc == nc, "coarse-face range of %d points", nc);
    nhang += v->hang_count[nc];
  }
  CHECK(nface == (int64_t)v->faces.size() && nhang == (int64_t)v->hangs.size(), "launch ranges miss faces");
  std::vector<int> seen(E, 0);
  for (int N = 1; N <= DG_VARP_MAXN; ++N)
    for (int lev = 0; lev < 2; ++lev)
      for (int i = v->first[N][lev]; i < v->first[N][lev] + v->count[N][lev]; ++i) {
        const int e = v->list[i];
        CHECK(e >= 0 && e < E, "list entry out of range");
        if (e < 0 || e >= E) continue;
        ++seen[e];
        CHECK(deg[e] + 1 == N && (geo[e].s == 1) == (lev == 1), "element %d listed in the wrong group", e);
      }
  for (int64_t e = 0; e < E; ++e) CHECK(seen[e] == 1, "element %lld listed %d times", (long long)e, seen[e]);
  dg_varp_destroy(v);
  return 0;
}

}  // namespace

int main() {
  std::mt19937 rng(15698);
  int meshes = 0;
  for (int nz = 1; nz <= 4; ++nz)
    for (int ny = 1; ny <= 4; ++ny)
      for (int nx = 1; nx <= 5; ++nx)
        for (int r = 0; r < 3; ++r) {
          std::vector<int> ref(nx * ny * nz);
          const double frac = r == 0 ? 0.0 : (r == 1 ? 0.3 : 0.7);
          for (int& x : ref) x = std::uniform_real_distribution<double>(0, 1)(rng) < frac;
          if (check_mesh(nx, ny, nz, ref, rng)) return 1;
          ++meshes;
        }
  // every cell refined
  std::vector<int> all(3 * 2 * 4, 1);
  if (check_mesh(3, 2, 4, all, rng)) return 1;
  if (fails) {
    printf("%d failures\n", fails);
    return 1;
  }
  printf("ok (%d meshes)\n", meshes + 1);
  return 0;
}
