// Internal declarations of the batched multi-mesh path.
#pragma once

#include "dg_internal.h"

// Per-mesh record in device memory.
struct DGBatchInst {
  DGTables tab;      // tables and mesh sizes of this mesh
  int N;             // p + 1
  int epb;           // elements per workgroup (tile) for this mesh's degree
  int64_t qoff;      // offset (doubles) of the mesh's block in Q / res / R
  double dt;         // time step of this mesh
};

// How the persistent grid shares out the work list.  Workgroups are dealt to
// the 8 XCDs round robin (workgroup w runs on XCD w % 8).  With xcd = 1 the
// list is cut into 8 contiguous parts of about equal work, bounds[x] ..
// bounds[x + 1], and the workgroups of XCD x walk part x round robin, so the
// items that run at the same time on one XCD are neighbours in the list (and
// their neighbour reads meet in that XCD's L2).  With xcd = 0 every
// workgroup walks the whole list round robin.
struct DGBatchSplit {
  int xcd;
  int bounds[9];
};

struct DGBatchLaunch {
  const DGBatchInst* inst;
  const int2* items;  // (mesh, first element)
  int nitems;
  unsigned grid;      // a multiple of 8 when split.xcd is set
  hipStream_t stream;
  int f32;
  DGBatchSplit split;
  // one launch per degree (DG_BATCH_PER_DEGREE): the items of point count N
  // are items[vbegin[N] .. vbegin[N] + vcount[N]), all with tile epb[N];
  // xcd: each XCD takes a contiguous part of them
  int per_degree;
  int xcd;
  int vbegin[DG_MAXN + 1], vcount[DG_MAXN + 1], epb[DG_MAXN + 1];
};

int dg_batch_tile_list(int N, int* out, int max);
// mode 0: RR = dQ/dt of every mesh (Qout unused); mode 1: RK stage,
// Qout = Qin + b res, res = RR in place.
int dg_batch_launch_stage(const DGBatchLaunch& L, int mode, const double* Qin, double* Qout, double* RR, double a,
                          double b, int first);
int dg_batch_blocks_per_cu(int f32);

// Shared with the single-mesh host code.
void dg_build_tables(int nx, int ny, int nz, int p, double gamma, const double L[3], DGTables* t, double* xi,
                     double* w);
extern const double kDgRKA[5];
extern const double kDgRKB[5];
int dg_set_error(int code, const char* fmt, ...);
