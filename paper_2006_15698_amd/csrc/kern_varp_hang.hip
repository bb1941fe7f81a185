// Hanging faces of the variable-degree mesh with refined cells: where a
// refined cell (eight children of half its size) meets an unrefined one,
// each fine element's face is a quarter of the coarse element's face.  Each
// quarter is integrated on the mortar of the hp setting (Sections I and
// III): the Gauss-Legendre rule of M = max(p_c, p_f) + 1 points per
// tangential direction on the fine face, both traces evaluated there (the
// coarse one at xi = (x^M_b + 2h - 1) / 2 on its half h of each tangential
// direction), the local Lax-Friedrichs flux formed once, and the flux
// integrated against each side's test functions with the quarter's area
// element.  With the collocated mass matrix divided out, the fine side's
// face term is the projection P[t][b] = l_t(x^M_b) W^M_b / w_t of the flux
// onto its face nodes, the coarse side's the sum over the four quarters of
// the projections l_t(xi_b) W^M_b / (2 w_t) per direction (the quarter's
// area).
//
// k_varp_hanging<NC>: one launch per coarse degree, one workgroup of four
// waves per coarse face:
//   1. the coarse trace at its face nodes into LDS, the five fields split
//      over the four waves (the coarse element is read once for its four
//      quarters; from the second RK stage of a call on, the traces come
//      from the trace buffer that the stage launches wrote);
//   2. wave q takes quarter q: the fine trace at its face nodes (into LDS
//      only where the fine degree is below the mortar's), both traces
//      interpolated to the mortar points, the flux, the fine side's
//      projection written to the face-flux buffer, the coarse side's into
//      LDS;
//   3. wave 0 sums the four quarters' coarse projections in the order
//      q = 0..3 and writes them to the buffer.

#include "dg_varp.h"
#include "stage_nb.h"

namespace dgdev {
namespace {

constexpr int kQuarters = 4;

struct HangLds {
  double gC[5 * 64];                 // coarse trace at its face nodes
  double gI[kQuarters][5 * 64];      // fine traces at their face nodes (NF < M)
  double gF[kQuarters][5 * 64];      // flux at the mortar points
  double gP[kQuarters][5 * 64];      // coarse projections of the quarters
};

// Quarter (q1, q2) of a coarse face of NC points on one wave, against a fine
// face of NF points; the mortar rule M = max(NC, NF) points on the fine face.
template <int NC, int NF, bool FT>
__device__ __forceinline__ void hang_quarter(const DGTables& tb, const DGVarpTabs* __restrict__ tabs,
                                             const DGVarpMesh& m, const DGVarpHang* __restrict__ H, int q,
                                             const double* __restrict__ Qin, HangLds& s, int lane) {
  constexpr int M = NC > NF ? NC : NF, M2 = M * M, C2 = NC * NC, F2 = NF * NF;
  const int d = H->d, q1 = q & 1, q2 = q >> 1;
  const bool cm = H->cminus != 0;   // the coarse element is on the -d side (its +d face)
  const double* cf = cm ? tabs->lm[NF] : tabs->lp[NF];
  const int64_t T = m.T;
  const int64_t sf = H->sf[q];
  double* gI = s.gI[q];
  double* gF = s.gF[q];
  const int b1 = lane % M, b2 = (lane < M2 ? lane : 0) / M;
  // the coarse side's interpolation rows of mortar point (b1, b2) on this
  // quarter, loaded while the state lines are in flight
  double r1[NC], r2[NC];
  {
    const double* I1 = tabs->hinterp[NC][M][q1];
    const double* I2 = tabs->hinterp[NC][M][q2];
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      r1[t] = I1[b1 * NC + t];
      r2[t] = I2[b2 * NC + t];
    }
  }
  double th[5];
  if (FT) {
    // the fine trace as its stage launch wrote it
    if (lane < F2) {
      const double* tf = m.tbuf + sf;
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        th[f] = tf[f * F2 + lane];
        if (NF < M) gI[f * 64 + lane] = th[f];
      }
    }
  } else if (lane < F2) {
    const double* qf = Qin + H->of[q];
    const int a = lane % NF, b = lane / NF;
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      double w[NF];
#pragma unroll
      for (int k = 0; k < NF; ++k) w[k] = qf[f * T + rt_node<NF>(d, k, a, b)];
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
        double x = 0.0;
#pragma unroll
        for (int t1 = 0; t1 < NC; ++t1) x = fma(r1[t1], s.gC[f * 64 + t1 + NC * t2], x);
        acc = fma(r2[t2], x, acc);
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
          double x = 0.0;
#pragma unroll
          for (int t1 = 0; t1 < NF; ++t1) x = fma(s1[t1], gI[f * 64 + t1 + NF * t2], x);
          acc = fma(s2[t2], x, acc);
        }
        tf[f] = acc;
      }
    }
    double fs[5];
    lf_flux(cm ? tc : tf, cm ? tf : tc, d, tb.gamma, tb.gm1, fs);
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      if (NF == M) m.fbuf[sf + f * M2 + lane] = fs[f];
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
        double x = 0.0;
#pragma unroll
        for (int c1 = 0; c1 < M; ++c1) x = fma(p1[c1], gF[f * 64 + c1 + M * c2], x);
        acc = fma(p2[c2], x, acc);
      }
      m.fbuf[sf + f * F2 + lane] = acc;
    }
  }
  if (lane < C2) {
    const int t1 = lane % NC, t2 = lane / NC;
    const double* P1 = tabs->hproj[NC][M][q1];
    const double* P2 = tabs->hproj[NC][M][q2];
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
        double x = 0.0;
#pragma unroll
        for (int c1 = 0; c1 < M; ++c1) x = fma(p1[c1], gF[f * 64 + c1 + M * c2], x);
        acc = fma(p2[c2], x, acc);
      }
      s.gP[q][f * 64 + lane] = acc;
    }
  }
}

// One coarse face of NC points and its four quarters on the workgroup.
template <int NC, bool FT>
__device__ __forceinline__ void hang_coarse(const DGTables& tb, const DGVarpTabs* __restrict__ tabs,
                                            const DGVarpMesh& m, const DGVarpHang* __restrict__ H,
                                            const double* __restrict__ Qin, HangLds& s, int wave, int lane) {
  constexpr int C2 = NC * NC;
  const int d = H->d;
  // 1. the coarse trace: field f on wave f % 4
  if (FT) {
    // as the coarse element's stage launch wrote it
    if (lane < C2) {
      for (int f = wave; f < 5; f += kQuarters) s.gC[f * 64 + lane] = m.tbuf[H->sc + f * C2 + lane];
    }
  } else if (lane < C2) {
    const double* cc = H->cminus ? tabs->lp[NC] : tabs->lm[NC];
    const double* qc = Qin + H->oc;
    const int a = lane % NC, b = lane / NC;
    for (int f = wave; f < 5; f += kQuarters) {
      double w[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) w[k] = qc[f * m.T + rt_node<NC>(d, k, a, b)];
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < NC; ++k) v = fma(cc[k], w[k], v);
      s.gC[f * 64 + lane] = v;
    }
  }
  __syncthreads();
  // 2. quarter q = wave
#define VARP_HANG(NF) \
  case NF: hang_quarter<NC, NF, FT>(tb, tabs, m, H, wave, Qin, s, lane); break;
  switch (H->nf[wave]) {   // uniform over the wave
    VARP_HANG(1) VARP_HANG(2) VARP_HANG(3) VARP_HANG(4) VARP_HANG(5) VARP_HANG(6) VARP_HANG(7) VARP_HANG(8)
    default: break;
  }
#undef VARP_HANG
  __syncthreads();
  // 3. the coarse side's sum over the quarters, in the order q = 0..3
  if (wave == 0 && lane < C2) {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      const int i = f * 64 + lane;
      m.fbuf[H->sc + f * C2 + lane] = ((s.gP[0][i] + s.gP[1][i]) + s.gP[2][i]) + s.gP[3][i];
    }
  }
}

// One launch per coarse degree present (coarse faces [begin, begin + grid)
// of that degree), so that each has its own register count (114-126 VGPRs
// up to NC = 6, against 144 for one kernel holding every degree).
template <int NC, bool FT>
__global__ void __launch_bounds__(64 * kQuarters) k_varp_hanging(const DGTables tb, const DGVarpMesh m,
                                                                  const double* __restrict__ Qin, int begin) {
  __shared__ HangLds s;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // one workgroup per coarse face: the grid has exactly the group's count
  const DGVarpHang* __restrict__ H = m.hangs + begin + blockIdx.x;
  hang_coarse<NC, FT>(tb, m.tabs, m, H, Qin, s, wave, lane);
}

}  // namespace
}  // namespace dgdev

int dg_launch_varp_hanging(hipStream_t stream, const DGTables& tb, const DGVarpMesh& m, const double* Qin, int nc,
                           int begin, int count, bool from_traces) {
  using namespace dgdev;
  if (count <= 0) return 0;
#define VARP_COARSE(NC)                                                                                       \
  case NC:                                                                                                    \
    if (from_traces)                                                                                          \
      hipLaunchKernelGGL((k_varp_hanging<NC, true>), dim3((unsigned)count), dim3(64 * kQuarters), 0, stream, tb, \
                         m, Qin, begin);                                                                      \
    else                                                                                                      \
      hipLaunchKernelGGL((k_varp_hanging<NC, false>), dim3((unsigned)count), dim3(64 * kQuarters), 0, stream,    \
                         tb, m, Qin, begin);                                                                  \
    break;
  switch (nc) {
    VARP_COARSE(1) VARP_COARSE(2) VARP_COARSE(3) VARP_COARSE(4) VARP_COARSE(5) VARP_COARSE(6) VARP_COARSE(7)
    VARP_COARSE(8)
    default: return (int)hipErrorInvalidValue;
  }
#undef VARP_COARSE
  return (int)hipGetLastError();
}
