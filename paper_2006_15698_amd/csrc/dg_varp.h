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
};

// A face between elements of different degrees: element a (its +d face)
// and its +d neighbour b (their -d face), with first nodes oa, ob; sa, sb
// the first double of the two sides' projected fluxes ([5][N_a^2],
// [5][N_b^2]) in the face-flux buffer.
struct DGVarpFace {
  int64_t oa, ob, sa, sb;
  int d;
  int code;            // (lo * (DG_VARP_MAXN + 1) + hi) * 2 + (1 if a has the lower degree)
};

// Mesh description read by every launch.
struct DGVarpMesh {
  const int64_t* off;      // first node of every element [E] (field stride T)
  const int64_t* slot;     // [E][6]: a face's projected flux in fbuf, -1 where conforming
  const int* list;         // elements grouped by degree, ascending inside a group
  const DGVarpTabs* tabs;
  const DGVarpFace* faces; // the mortar faces, grouped by code
  double* fbuf;            // projected fluxes of the mortar faces
  int64_t T;               // total nodes
  int nx, ny, nz;
  int nfaces;
};

// Launch one stage (mode 0: RR = dQ/dt; 1: LSERK45 stage Qin -> Qout with
// res = RR in place; 2: the first stage) over the `count` elements of degree
// N - 1 listed from list[first].  Reads the mortar fluxes that
// dg_launch_varp_mortar wrote for the same Qin.
int dg_launch_varp(hipStream_t stream, int N, const DGTables& tb, const DGVarpMesh& m, int first, int count,
                   const double* Qin, double* Qout, double* RR, int mode, double a, double b, double dt);
// The flux of every mortar face of Qin, projected onto both sides' face
// nodes, into m.fbuf.
int dg_launch_varp_mortar(hipStream_t stream, const DGTables& tb, const DGVarpMesh& m, const double* Qin);
// Elements per workgroup of the variable-degree kernel for N points.
int dg_varp_epb(int N);
