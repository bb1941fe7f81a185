// Hanging faces of the variable-degree mesh with refined cells: where a
// refined cell (eight children of half its size) meets an unrefined one,
// each fine element's face is a quarter of the coarse element's face.  The
// sub-face is integrated on the mortar of the hp setting (Sections I and
// III): the Gauss-Legendre rule of M = max(p_c, p_f) + 1 points per
// tangential direction on the fine face, both traces evaluated there (the
// coarse one at xi = (x^M_b + 2h - 1) / 2 on its half h of each tangential
// direction), the local Lax-Friedrichs flux formed once, and the flux
// integrated against each side's test functions with the sub-face's area
// element.  With the collocated mass matrix divided out, the fine side's
// face term is the projection P[t][b] = l_t(x^M_b) W^M_b / w_t of the
// flux onto its face nodes, the coarse side's the projection
// l_t(xi_b) W^M_b / (2 w_t) per direction (the quarter's area) into this
// quarter's block; the coarse element's kernel sums its four quarters.
//
// k_varp_hanging: one wave per sub-face (sub-faces grouped by degree pair):
//   both traces at their face nodes (the fine one into LDS only where the
//   fine degree is below the mortar's), both interpolated to the mortar
//   points, the flux, the two projections written into the face-flux
//   buffer.

#include "dg_varp.h"
#include "stage_nb.h"

namespace dgdev {
namespace {

// One hanging sub-face on one wave: the coarse side NC points, the fine side
// NF points per direction, the mortar rule M = max(NC, NF) points on the fine
// face (the fine element's own coordinate; on the coarse face the quarter
// (q1, q2)).  g: this wave's LDS region [5][64] coarse trace, [5][64] fine
// trace, [5][64] flux.
template <int NC, int NF>
__device__ __forceinline__ void hang_face(const DGTables& tb, const DGVarpTabs* __restrict__ tabs,
                                          const DGVarpMesh& m, const DGVarpHang& H,
                                          const double* __restrict__ Qin, double* g, int lane) {
  constexpr int M = NC > NF ? NC : NF, M2 = M * M, C2 = NC * NC, F2 = NF * NF;
  const int d = H.d;
  const bool cm = H.cminus != 0;   // the coarse element is on the -d side (its +d face)
  const double* cc = cm ? tabs->lp[NC] : tabs->lm[NC];
  const double* cf = cm ? tabs->lm[NF] : tabs->lp[NF];
  const int64_t T = m.T;
  double* gC = g;          // coarse trace at its face nodes
  double* gI = g + 320;    // fine trace at its face nodes (NF < M)
  double* gF = g + 640;    // flux at the mortar points
  const int b1 = lane % M, b2 = (lane < M2 ? lane : 0) / M;
  // the coarse side's interpolation rows of mortar point (b1, b2) on this
  // quarter, loaded while the state lines are in flight
  double r1[NC], r2[NC];
  {
    const double* I1 = tabs->hinterp[NC][M][H.q1];
    const double* I2 = tabs->hinterp[NC][M][H.q2];
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      r1[t] = I1[b1 * NC + t];
      r2[t] = I2[b2 * NC + t];
    }
  }
  if (lane < C2) {
    const double* q = Qin + H.oc;
    const int a = lane % NC, b = lane / NC;
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      double w[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) w[k] = q[f * T + rt_node<NC>(d, k, a, b)];
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < NC; ++k) v = fma(cc[k], w[k], v);
      gC[f * 64 + lane] = v;
    }
  }
  double th[5];
  if (lane < F2) {
    const double* q = Qin + H.of;
    const int a = lane % NF, b = lane / NF;
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      double w[NF];
#pragma unroll
      for (int k = 0; k < NF; ++k) w[k] = q[f * T + rt_node<NF>(d, k, a, b)];
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < NF; ++k) v = fma(cf[k], w[k], v);
      th[f] = v;
      if (NF < M) gI[f * 64 + lane] = v;
    }
  }
  __syncwarp();
  if (lane < M2) {
    double tc[5], tf[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      double acc = 0.0;
#pragma unroll
      for (int t2 = 0; t2 < NC; ++t2) {
        double s = 0.0;
#pragma unroll
        for (int t1 = 0; t1 < NC; ++t1) s = fma(r1[t1], gC[f * 64 + t1 + NC * t2], s);
        acc = fma(r2[t2], s, acc);
      }
      tc[f] = acc;
    }
    if (NF == M) {
#pragma unroll
      for (int f = 0; f < 5; ++f) tf[f] = th[f];
    } else {
      const double* I = tabs->interp[NF][M];
      double s1[NF], s2[NF];
#pragma unroll
      for (int t = 0; t < NF; ++t) {
        s1[t] = I[b1 * NF + t];
        s2[t] = I[b2 * NF + t];
      }
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        double acc = 0.0;
#pragma unroll
        for (int t2 = 0; t2 < NF; ++t2) {
          double s = 0.0;
#pragma unroll
          for (int t1 = 0; t1 < NF; ++t1) s = fma(s1[t1], gI[f * 64 + t1 + NF * t2], s);
          acc = fma(s2[t2], s, acc);
        }
        tf[f] = acc;
      }
    }
    double fs[5];
    lf_flux(cm ? tc : tf, cm ? tf : tc, d, tb.gamma, tb.gm1, fs);
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      if (NF == M) m.fbuf[H.sf + f * M2 + lane] = fs[f];
      gF[f * 64 + lane] = fs[f];
    }
  }
  __syncwarp();
  if (NF < M && lane < F2) {
    const double* P = tabs->proj[NF][M];
    const int t1 = lane % NF, t2 = lane / NF;
    double p1[M], p2[M];
#pragma unroll
    for (int b = 0; b < M; ++b) {
      p1[b] = P[t1 * M + b];
      p2[b] = P[t2 * M + b];
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      double acc = 0.0;
#pragma unroll
      for (int c2 = 0; c2 < M; ++c2) {
        double s = 0.0;
#pragma unroll
        for (int c1 = 0; c1 < M; ++c1) s = fma(p1[c1], gF[f * 64 + c1 + M * c2], s);
        acc = fma(p2[c2], s, acc);
      }
      m.fbuf[H.sf + f * F2 + lane] = acc;
    }
  }
  if (lane < C2) {
    const int t1 = lane % NC, t2 = lane / NC;
    const double* P1 = tabs->hproj[NC][M][H.q1];
    const double* P2 = tabs->hproj[NC][M][H.q2];
    double p1[M], p2[M];
#pragma unroll
    for (int b = 0; b < M; ++b) {
      p1[b] = P1[t1 * M + b];
      p2[b] = P2[t2 * M + b];
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      double acc = 0.0;
#pragma unroll
      for (int c2 = 0; c2 < M; ++c2) {
        double s = 0.0;
#pragma unroll
        for (int c1 = 0; c1 < M; ++c1) s = fma(p1[c1], gF[f * 64 + c1 + M * c2], s);
        acc = fma(p2[c2], s, acc);
      }
      m.fbuf[H.sc + f * C2 + lane] = acc;
    }
  }
}

constexpr int kHangWaves = 4;

__global__ void __launch_bounds__(64 * kHangWaves) k_varp_hanging(const DGTables tb, const DGVarpMesh m,
                                                                   const double* __restrict__ Qin) {
  __shared__ double sg[kHangWaves][960];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int hi = blockIdx.x * kHangWaves + wave;
  if (hi >= m.nhangs) return;   // whole waves: no workgroup barrier below
  const DGVarpHang H = m.hangs[hi];
  const DGVarpTabs* __restrict__ tabs = m.tabs;
  double* g = sg[wave];
#define VARP_HANG(NC, NF) \
  case (NC) * (DG_VARP_MAXN + 1) + (NF): hang_face<NC, NF>(tb, tabs, m, H, Qin, g, lane); break;
#define VARP_HANG_ROW(NC) \
  VARP_HANG(NC, 1) VARP_HANG(NC, 2) VARP_HANG(NC, 3) VARP_HANG(NC, 4) VARP_HANG(NC, 5) VARP_HANG(NC, 6) \
  VARP_HANG(NC, 7) VARP_HANG(NC, 8)
  switch (H.nc * (DG_VARP_MAXN + 1) + H.nf) {   // uniform over the wave
    VARP_HANG_ROW(1) VARP_HANG_ROW(2) VARP_HANG_ROW(3) VARP_HANG_ROW(4)
    VARP_HANG_ROW(5) VARP_HANG_ROW(6) VARP_HANG_ROW(7) VARP_HANG_ROW(8)
    default: break;
  }
#undef VARP_HANG_ROW
#undef VARP_HANG
}

}  // namespace
}  // namespace dgdev

int dg_launch_varp_hanging(hipStream_t stream, const DGTables& tb, const DGVarpMesh& m, const double* Qin) {
  using namespace dgdev;
  if (m.nhangs <= 0) return 0;
  const unsigned grid = (unsigned)((m.nhangs + kHangWaves - 1) / kHangWaves);
  hipLaunchKernelGGL(k_varp_hanging, dim3(grid), dim3(64 * kHangWaves), 0, stream, tb, m, Qin);
  return (int)hipGetLastError();
}
