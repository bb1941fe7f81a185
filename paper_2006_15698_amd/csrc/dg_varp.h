// Internal declarations of the variable-degree entry points (dg_varp_* in
// dg.h): the mortar tables and the launch arguments shared by the host code
// (varp_api.cpp) and the kernels (kern_varp.hip).
#pragma once

#include "dg_internal.h"

// Largest supported points per direction (p = 0..7, as for one degree).
#define DG_VARP_MAXN DG_MAXN

// Tables of the mortar faces, in device memory (the workspace), read with
// indices that are uniform over a face.  Index n below is a point count
// N = p + 1 in 1..DG_VARP_MAXN (slot 0 unused).
struct DGVarpTabs {
  // l^n_m(-1), l^n_m(+1): a degree-(n-1) element's trace on its -/+ face
  // (the same values as DGTables::lm/lp of that degree)
  double lm[DG_VARP_MAXN + 1][DG_VARP_MAXN];
  double lp[DG_VARP_MAXN + 1][DG_VARP_MAXN];
  // interp[n][m][b * n + t] = l^n_t(x^m_b): the degree-(n-1) basis at the
  // m Gauss-Legendre points of the mortar rule (m > n)
  double interp[DG_VARP_MAXN + 1][DG_VARP_MAXN + 1][DG_VARP_MAXN * DG_VARP_MAXN];
  // proj[n][m][t * m + b] = l^n_t(x^m_b) W^m_b / w^n_t: the mortar rule's
  // weights times the basis, over the element's own face weights (the
  // surface integral on the mortar, lifted by the diagonal mass matrix)
  double proj[DG_VARP_MAXN + 1][DG_VARP_MAXN + 1][DG_VARP_MAXN * DG_VARP_MAXN];
  // the same on one half of a coarse face (h = 0: xi in [-1, 0], h = 1:
  // [0, 1]), at xi = (x^m_b + 2h - 1) / 2, for m >= n; the projection
  // carries the half's factor 1/2 (a fine face is a quarter of the coarse
  // face: 1/2 per direction)
  double hinterp[DG_VARP_MAXN + 1][DG_VARP_MAXN + 1][2][DG_VARP_MAXN * DG_VARP_MAXN];
  double hproj[DG_VARP_MAXN + 1][DG_VARP_MAXN + 1][2][DG_VARP_MAXN * DG_VARP_MAXN];
};

// A face between elements of the same size and different degrees: element
// a (its +d face) and its +d neighbour b (their -d face), with first nodes
// oa, ob; sa, sb the first double of the two sides' projected fluxes
// ([5][N_a^2], [5][N_b^2]) in the face-flux buffer.
struct DGVarpFace {
  int64_t oa, ob, sa, sb;
  int d;
  int code;            // (lo * (DG_VARP_MAXN + 1) + hi) * 2 + (1 if a has the lower degree)
};

// A coarse face against the four fine faces of a refined neighbour cell
// (hanging faces): quarter q = 2 q2 + q1 (q1, q2 the halves along the two
// tangential axes in increasing order) is the whole face of fine element
// q.  oc, of[q]: first nodes; sc: the coarse side's summed projection
// ([5][N_c^2]); sf[q]: fine element q's ([5][N_f^2]); cminus: the coarse
// element is on the -d side (its +d face).
struct DGVarpHang {
  int64_t oc, sc;
  int64_t of[4], sf[4];
  int nf[4];
  int d, nc, cminus, pad;
};

// What a face of an element takes its flux from: the low two bits of
// DGVarpMesh::face, the rest (face >> 2) the place it names.
enum {
  DG_FACE_CONFORMING = 0,  // same size and degree: the neighbour's first node
  DG_FACE_MORTAR = 1       // the projected flux [5][N^2] in fbuf (a face between
                           // degrees, or either side of a hanging face)
};

// Mesh description read by every launch.
struct DGVarpMesh {
  const int64_t* off;      // first node of every element [E] (field stride T)
  const int64_t* face;     // [E][6]: (place << 2) | DG_FACE_* of face 2d + side
  const int* list;         // elements grouped by (degree, size), each group in visiting order
  const DGVarpTabs* tabs;
  const DGVarpFace* faces; // the mortar faces, grouped by code
  const DGVarpHang* hangs; // the coarse faces with hanging faces, grouped by degree
  double* fbuf;            // projected fluxes of the mortar and hanging faces
  double* tbuf;            // the elements' own traces on those faces, at the same
                           // places as their fluxes in fbuf ([5][N^2] each)
  int64_t T;               // total nodes
  int nfaces, nhangs;
};

// Launch one stage (mode 0: RR = dQ/dt; 1: LSERK45 stage Qin -> Qout with
// res = RR in place; 2: the first stage) over the `count` elements of N
// points and one size listed from list[first] (tb: that size's tables).
// Reads the mortar and hanging fluxes written for the same Qin.  traces
// (modes 1, 2): also write every element's trace of Qout on its faces that
// take their flux from fbuf into m.tbuf, for the next stage's face launches.
int dg_launch_varp(hipStream_t stream, int N, const DGTables& tb, const DGVarpMesh& m, int first, int count,
                   const double* Qin, double* Qout, double* RR, int mode, double a, double b, double dt, bool traces);
// The flux of the mortar faces [begin, begin + count) of Qin, all between
// degrees lo - 1 < hi - 1 (point counts lo, hi), projected onto both sides'
// face nodes, into m.fbuf.  from_traces: both sides' traces from m.tbuf
// (written by the stage launches that produced Qin) instead of from Qin.
int dg_launch_varp_mortar(hipStream_t stream, const DGTables& tb, const DGVarpMesh& m, const double* Qin, int lo,
                          int hi, int begin, int count, bool from_traces);
// The flux of every hanging face of Qin, projected onto the fine sides'
// face nodes and (summed over the four quarters) the coarse side's, into
// m.fbuf (the coarse faces [begin, begin + count), all of nc points).
// from_traces as for the mortar launch.
int dg_launch_varp_hanging(hipStream_t stream, const DGTables& tb, const DGVarpMesh& m, const double* Qin, int nc,
                           int begin, int count, bool from_traces);
// Elements per workgroup of the variable-degree kernel for N points.
int dg_varp_epb(int N);

namespace dgdev {
// Node of a degree-(n-1) element: index m along direction d, tangential
// point (a, b) (lower tangential axis a), as tnode with a runtime d.
template <int NN>
__device__ __forceinline__ int rt_node(int d, int m, int a, int b) {
  if (d == 0) return m + NN * (a + NN * b);
  if (d == 1) return a + NN * (m + NN * b);
  return a + NN * (b + NN * m);
}

}  // namespace dgdev
