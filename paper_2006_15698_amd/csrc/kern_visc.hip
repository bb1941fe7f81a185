// Viscous (Navier-Stokes) terms on the collocated Gauss-Legendre basis:
// Bassi & Rebay's first scheme (BR1).
//
// The paper names the viscous formulation of its CPU code (Section III,
// Fig. 2) without printing it; the reading taken (constant mu, Stokes'
// hypothesis, Fourier conduction at constant Prandtl number, gas constant 1
// so T = p / rho):
//   theta_d = grad_d of the primitive quantities P = (u, v, w, T), the weak
//             derivative of their nodal interpolants with the central mean
//             of the two sides' traces on every face;
//   F_v^d   = (0, tau_1d, tau_2d, tau_3d, u_k tau_kd + kappa dT/dx_d),
//             tau_kd = mu (du_k/dx_d + du_d/dx_k - 2/3 delta_kd div u),
//             evaluated at the nodes;
//   dQ/dt  += the weak derivative of F_v^d's nodal interpolant with the
//             central mean of the two sides' traces, summed over d.
// Both weak derivatives have the form, along the d-line of node i (the mass
// matrix divided out, as in the inviscid stage):
//   (2/h_d) [ -sum_a Dh[i][a] X_a + l_i(+1)/w_i {X}_+ - l_i(-1)/w_i {X}_- ].
//
// Two launches per right-hand side, one workgroup per element (elements
// visited in the neighbour-read stage's order: pencils, each XCD a
// contiguous part), one thread per node:
//   k_visc_flux  Q -> F_v at every node (12 values: 4 per direction);
//                the neighbours' primitive traces are interpolated from
//                their state in the same launch (on y/z-faces two points per
//                16-byte load); with RATE it writes the inviscid rate R of
//                the standard form too, from the same neighbour loads;
//   k_visc_apply F_v -> the viscous rate, added to the inviscid rate R (of
//                the flux launch, or of the split-form or FP32 kernel)
//                (MODE 0), or combined with it into the LSERK45 update of Q
//                and res in place (MODE 1, MODE 2 for the first stage: no
//                launch reads another element's Q here).

#include "dg_internal.h"
#include "stage_fp64.h"
#include "stage_nb.h"

namespace {

template <int N>
struct VCfg {
  static constexpr int N2 = N * N;
  static constexpr int N3 = N * N * N;
  static constexpr int NT = N3 <= 64 ? 64 : (N3 + 63) / 64 * 64;
  static constexpr int NW = NT / 64;
  // face phase: LPF lanes per face, FPW faces per wave (the two faces of
  // one direction share a wave when a face fits half a wave, so the
  // direction is uniform over the wave and static inside the loads),
  // NSLOT wave-sized slots per element
  static constexpr int LPF = N2 <= 32 ? 32 : 64;
  static constexpr int FPW = 64 / LPF;
  static constexpr int NSLOT = 6 / FPW;
};

// The flux launch's neighbour-trace phase: WX wave-sized slots for the x-face
// points (one per lane), then slots for the y/z-face point pairs (NYZ pairs,
// H per row).
template <int N>
struct PairCfg {
  // a pair needs rows of two points; at N = 7, 8 the pair slots would
  // leave waves of the workgroup idle in this phase (p = 6: 2.6% slower)
  static constexpr bool PAIRS = N >= 2 && N <= 6;
  static constexpr int H = (N + 1) / 2;
  static constexpr int NYZ = 4 * N * H;
  static constexpr int WX = (2 * N * N + 63) / 64;
  static constexpr int SLOTS = WX + (NYZ + 63) / 64;
};

// Face and tangential point of lane `lane` in face slot `s`; false for the
// lanes past the face's points.
template <int N>
__device__ __forceinline__ bool face_lane(int s, int lane, int& face, int& pt) {
  face = s * VCfg<N>::FPW + lane / VCfg<N>::LPF;
  pt = lane % VCfg<N>::LPF;
  return pt < VCfg<N>::N2;
}

// (u, v, w, T) of a conserved state, T = p / rho with Eq. (3)'s pressure.
__device__ __forceinline__ void primitive(const double* q, double gm1, double* P) {
  const double r = dgdev::recip(q[0]);
  P[0] = q[1] * r;
  P[1] = q[2] * r;
  P[2] = q[3] * r;
  const double ke = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) * r;
  P[3] = gm1 * (q[4] - ke) * r;
}

// Tangential point index (lower tangential axis fastest) and position
// along direction d of node (i, j, k).
template <int N>
__device__ __forceinline__ void line_of(int d, int i, int j, int k, int& m, int& pt) {
  if (d == 0) { m = i; pt = j + N * k; }
  else if (d == 1) { m = j; pt = i + N * k; }
  else { m = k; pt = i + N * j; }
}

// BR1 weak derivative along the d-line through node position m0 of the
// field X (LDS, N^3 values): own traces from the line, neighbour traces
// tm (on the -d face) and tp (on the +d face) given.
template <int N>
__device__ __forceinline__ double br1_line(const DGTables& tb, const double* X, int d, int m0, int pt, double tm,
                                           double tp) {
  double own_m = 0.0, own_p = 0.0, vol = 0.0;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    const double x = X[dgdev::tnode<N>(d, a, pt)];
    own_m = fma(tb.lm[a], x, own_m);
    own_p = fma(tb.lp[a], x, own_p);
    vol = fma(tb.Dh[m0 * N + a], x, vol);
  }
  const double hat_m = 0.5 * (own_m + tm);
  const double hat_p = 0.5 * (own_p + tp);
  return tb.sc[d] * (tb.liftp[m0] * hat_p - tb.liftm[m0] * hat_m - vol);
}

// A neighbour's primitive trace on our face point pt of direction D: its
// -D face (s = 1, our +D face) or its +D face (s = 0), from its state at q
// (field stride fs), summed over its normal line; with CONS also its
// conserved trace from the same loads (the FMA chain of line_trace).
template <int N, int D, bool CONS>
__device__ __forceinline__ void prim_trace(const DGTables& tb, const double* __restrict__ q, int64_t fs, int s,
                                           int pt, double* acc, double* cons) {
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = 0.0;
  if (CONS) {
#pragma unroll
    for (int f = 0; f < 5; ++f) cons[f] = 0.0;
  }
#pragma unroll
  for (int m = 0; m < N; ++m) {
    const int node = dgdev::tnode<N>(D, m, pt);
    double v[5], p[4];
#pragma unroll
    for (int f = 0; f < 5; ++f) v[f] = q[f * fs + node];
    primitive(v, tb.gm1, p);
    const double wgt = s ? tb.lm[m] : tb.lp[m];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = fma(wgt, p[c], acc[c]);
    if (CONS) {
#pragma unroll
      for (int f = 0; f < 5; ++f) cons[f] = fma(wgt, v[f], cons[f]);
    }
  }
}

// prim_trace for the two points a0, a0 + 1 of row b of a y- or z-face
// (tangential index a + N b): their normal-line nodes a + m sm + b sb
// (sm, sb = N, N^2 for y and N^2, N for z) are next to each other in memory
// at every position m, so one 16-byte load (a multi-dword access needs only
// dword alignment) brings a field's value for both.  Per point the FMA
// chains of prim_trace.
template <int N, bool CONS>
__device__ __forceinline__ void prim_trace_pair(const DGTables& tb, const double* __restrict__ q, int64_t fs, int s,
                                                int sm, int node0, double (*acc)[4], double (*cons)[5]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[h][c] = 0.0;
    if (CONS) {
#pragma unroll
      for (int f = 0; f < 5; ++f) cons[h][f] = 0.0;
    }
  }
#pragma unroll
  for (int m = 0; m < N; ++m) {
    const int node = node0 + m * sm;
    double2 w[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) __builtin_memcpy(&w[f], q + f * fs + node, 16);
    const double wgt = s ? tb.lm[m] : tb.lp[m];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double v[5], p[4];
#pragma unroll
      for (int f = 0; f < 5; ++f) v[f] = h ? w[f].y : w[f].x;
      primitive(v, tb.gm1, p);
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[h][c] = fma(wgt, p[c], acc[h][c]);
      if (CONS) {
#pragma unroll
        for (int f = 0; f < 5; ++f) cons[h][f] = fma(wgt, v[f], cons[h][f]);
      }
    }
  }
}

// Local Lax-Friedrichs flux at face point pt of face 2D + s from the
// element's own trace (interpolated from its state S in LDS) and the
// neighbour's (in H, overwritten with the flux).
template <int N, int D>
__device__ __forceinline__ void face_flux(const DGTables& tb, const double (*S)[VCfg<N>::N3],
                                          double (*H)[VCfg<N>::N2], int s, int pt) {
  double own[5], qm[5], qp[5], fl[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    own[f] = dgdev::line_trace<N>(S[f], s ? tb.lp : tb.lm, D, pt);
    const double nb = H[f][pt];
    qm[f] = s ? own[f] : nb;
    qp[f] = s ? nb : own[f];
  }
  dgdev::lf_flux_d<D>(qm, qp, tb.gamma, tb.gm1, fl);
#pragma unroll
  for (int f = 0; f < 5; ++f) H[f][pt] = fl[f];
}

// A neighbour's trace of its direction-D viscous flux (4 values) on our
// face point pt, as prim_trace.
template <int N, int D>
__device__ __forceinline__ void flux_trace(const DGTables& tb, const double* __restrict__ fv, int64_t fs, int s,
                                           int pt, double* acc) {
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = 0.0;
#pragma unroll
  for (int m = 0; m < N; ++m) {
    const int node = dgdev::tnode<N>(D, m, pt);
    const double wgt = s ? tb.lm[m] : tb.lp[m];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = fma(wgt, fv[(D * 4 + c) * fs + node], acc[c]);
  }
}

// flux_trace for a pair of points of a y- or z-face (direction d), as
// prim_trace_pair.
template <int N>
__device__ __forceinline__ void flux_trace_pair(const DGTables& tb, const double* __restrict__ fv, int64_t fs, int s,
                                                int d, int sm, int node0, double (*acc)[4]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[h][c] = 0.0;
  }
#pragma unroll
  for (int m = 0; m < N; ++m) {
    const int node = node0 + m * sm;
    const double wgt = s ? tb.lm[m] : tb.lp[m];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double2 w;
      __builtin_memcpy(&w, fv + (d * 4 + c) * fs + node, 16);
      acc[0][c] = fma(wgt, w.x, acc[0][c]);
      acc[1][c] = fma(wgt, w.y, acc[1][c]);
    }
  }
}

// RATE: the inviscid (Euler) rate of the standard form as well, into R: the
// neighbours' conserved traces come from the loads of their primitive
// traces, the element's own from its state in LDS; the operations and their
// order are those of the fused Euler stage (same traces, Lax-Friedrichs
// flux, pointwise flux staged per direction, contraction and lift), so R
// equals the neighbour-read kernel's rate.
template <int N, bool RATE>
__global__ void __launch_bounds__(VCfg<N>::NT)
k_visc_flux(DGTables tb, const double* __restrict__ Q, double* __restrict__ Fv, double* __restrict__ R, double mu,
            double kappa, DGOrder ord) {
  constexpr int N2 = VCfg<N>::N2, N3 = VCfg<N>::N3, NT = VCfg<N>::NT;
  constexpr int RN3 = RATE ? N3 : 1, RN2 = RATE ? N2 : 1;
  __shared__ double P[4][N3];
  __shared__ double Tn[6][4][N2];   // face 2d + s: neighbour's trace (s = 0: -d face, 1: +d face)
  __shared__ double S[5][RN3];      // RATE: the state, then one direction's pointwise Euler flux
  __shared__ double H[6][5][RN2];   // RATE: the neighbour's conserved trace, then the face flux
  // the element of this workgroup in the visiting order (pencils, XCD chunks)
  int e, ne;
  dgdev::block_elements<1>(tb, ord, blockIdx.x, gridDim.x, e, ne);
  const int t = threadIdx.x;
  const int64_t fs = (int64_t)tb.E * N3;
  double q[5];   // with RATE: the node's state, read back from S after the first barrier
  if constexpr (N3 >= 2) {
    // two nodes per lane and 16-byte load (dword alignment suffices; at odd
    // N^3 the last pair overlaps the one before it)
    constexpr int NP = (N3 + 1) / 2;
    if (t < NP) {
      const int n0 = 2 * t < N3 - 2 ? 2 * t : N3 - 2;
      double2 w[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) __builtin_memcpy(&w[f], Q + f * fs + (int64_t)e * N3 + n0, 16);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double v[5], p[4];
#pragma unroll
        for (int f = 0; f < 5; ++f) v[f] = h ? w[f].y : w[f].x;
        primitive(v, tb.gm1, p);
#pragma unroll
        for (int c = 0; c < 4; ++c) P[c][n0 + h] = p[c];
        if (RATE) {
#pragma unroll
          for (int f = 0; f < 5; ++f) S[f][RATE ? n0 + h : 0] = v[f];
        }
      }
    }
  } else if (t < N3) {
    double p[4];
#pragma unroll
    for (int f = 0; f < 5; ++f) q[f] = Q[f * fs + (int64_t)e * N3 + t];
    primitive(q, tb.gm1, p);
#pragma unroll
    for (int c = 0; c < 4; ++c) P[c][t] = p[c];
    if (RATE) {
#pragma unroll
      for (int f = 0; f < 5; ++f) S[f][RATE ? t : 0] = q[f];
    }
  }
  const int wave = t >> 6, lane = t & 63;
  using PC = PairCfg<N>;
  if constexpr (!PC::PAIRS) {
    for (int sl = wave; sl < VCfg<N>::NSLOT; sl += VCfg<N>::NW) {
      int face, pt;
      if (face_lane<N>(sl, lane, face, pt)) {
        const int s = face & 1;
        const int en = dgdev::neighbour(tb.nx, tb.ny, tb.nz, e, face >> 1, s ? 1 : -1);
        double acc[4], cons[5];
        switch (face >> 1) {   // uniform over the wave
          case 0: prim_trace<N, 0, RATE>(tb, Q + (int64_t)en * N3, fs, s, pt, acc, cons); break;
          case 1: prim_trace<N, 1, RATE>(tb, Q + (int64_t)en * N3, fs, s, pt, acc, cons); break;
          default: prim_trace<N, 2, RATE>(tb, Q + (int64_t)en * N3, fs, s, pt, acc, cons); break;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) Tn[face][c][pt] = acc[c];
        if (RATE) {
#pragma unroll
          for (int f = 0; f < 5; ++f) H[face][f][RATE ? pt : 0] = cons[f];
        }
      }
    }
  } else for (int sl = wave; sl < PC::SLOTS; sl += VCfg<N>::NW) {
    if (sl < PC::WX) {
      // x-faces: one point per lane
      const int it = sl * 64 + lane;
      if (it < 2 * N2) {
        const int s = it >= N2, pt = it - s * N2, face = s;
        const int en = dgdev::neighbour(tb.nx, tb.ny, tb.nz, e, 0, s ? 1 : -1);
        double acc[4], cons[5];
        prim_trace<N, 0, RATE>(tb, Q + (int64_t)en * N3, fs, s, pt, acc, cons);
#pragma unroll
        for (int c = 0; c < 4; ++c) Tn[face][c][pt] = acc[c];
        if (RATE) {
#pragma unroll
          for (int f = 0; f < 5; ++f) H[face][f][RATE ? pt : 0] = cons[f];
        }
      }
    } else {
      // y- and z-faces: two points of a row per lane (rows of odd length
      // end in a pair that overlaps the one before it; both write the same
      // values for the shared point)
      const int it = (sl - PC::WX) * 64 + lane;
      if (it < PC::NYZ) {
        const int qf = it / (N * PC::H), r = it - qf * (N * PC::H);
        const int b = r / PC::H, c2 = r - b * PC::H;
        const int a0 = 2 * c2 < N - 2 ? 2 * c2 : N - 2;
        const int d = 1 + (qf >> 1), s = qf & 1, face = 2 * d + s;
        const int sm = d == 1 ? N : N2, sb = d == 1 ? N2 : N;
        const int en = dgdev::neighbour(tb.nx, tb.ny, tb.nz, e, d, s ? 1 : -1);
        double acc[2][4], cons[2][5];
        prim_trace_pair<N, RATE>(tb, Q + (int64_t)en * N3, fs, s, sm, a0 + b * sb, acc, cons);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int pt = a0 + h + N * b;
#pragma unroll
          for (int c = 0; c < 4; ++c) Tn[face][c][pt] = acc[h][c];
          if (RATE) {
#pragma unroll
            for (int f = 0; f < 5; ++f) H[face][f][RATE ? pt : 0] = cons[h][f];
          }
        }
      }
    }
  }
  __syncthreads();
  if constexpr (RATE) {
    if (N3 >= 2 && t < N3) {
#pragma unroll
      for (int f = 0; f < 5; ++f) q[f] = S[f][t];
    }
    // the face fluxes (each lane rewrites only its own points of H)
    for (int sl = wave; sl < VCfg<N>::NSLOT; sl += VCfg<N>::NW) {
      int face, pt;
      if (face_lane<N>(sl, lane, face, pt)) {
        switch (face >> 1) {
          case 0: face_flux<N, 0>(tb, S, H[face], face & 1, pt); break;
          case 1: face_flux<N, 1>(tb, S, H[face], face & 1, pt); break;
          default: face_flux<N, 2>(tb, S, H[face], face & 1, pt); break;
        }
      }
    }
  } else if (t >= N3) {
    return;
  }
  const bool node = t < N3;
  const int i = t % N, j = (t / N) % N, k = t / N2;
  const int64_t g = (int64_t)e * N3 + t;
  if (node) {
    double th[3][4];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int m0, pt;
      line_of<N>(d, i, j, k, m0, pt);
#pragma unroll
      for (int c = 0; c < 4; ++c) th[d][c] = br1_line<N>(tb, P[c], d, m0, pt, Tn[2 * d][c][pt], Tn[2 * d + 1][c][pt]);
    }
    const double u[3] = {P[0][t], P[1][t], P[2][t]};
    const double div = th[0][0] + th[1][1] + th[2][2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double en = kappa * th[d][3];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        double tau = mu * (th[d][kk] + th[kk][d]);
        if (kk == d) tau = tau - (2.0 / 3.0) * mu * div;
        Fv[(d * 4 + kk) * fs + g] = tau;
        en = en + u[kk] * tau;
      }
      Fv[(d * 4 + 3) * fs + g] = en;
    }
  }
  if (!RATE) return;
  // Euler volume term: per direction the pointwise flux into S (free once
  // every face flux is formed), then the contraction along the node's line
  // and the lift of the two face fluxes on it
  double rinv = 0.0, pr = 0.0;
  if (node) {
    rinv = dgdev::recip(q[0]);
    pr = tb.gm1 * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) * rinv);
  }
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    __syncthreads();   // S (state, or the previous direction's flux) is no longer read
    if (node) {
      const double ud = q[1 + d] * rinv;
      S[0][RATE ? t : 0] = q[1 + d];
      S[1][RATE ? t : 0] = q[1] * ud + (d == 0 ? pr : 0.0);
      S[2][RATE ? t : 0] = q[2] * ud + (d == 1 ? pr : 0.0);
      S[3][RATE ? t : 0] = q[3] * ud + (d == 2 ? pr : 0.0);
      S[4][RATE ? t : 0] = (q[4] + pr) * ud;
    }
    __syncthreads();
    if (node) {
      int m, pt;
      line_of<N>(d, i, j, k, m, pt);
      const double sc = tb.sc[d];
      const double lfm = tb.liftm[m], lfp = tb.liftp[m];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        double sm = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) sm = fma(tb.Dh[m * N + a], S[f][RATE ? dgdev::tnode<N>(d, a, pt) : 0], sm);
        sm = fma(lfm, H[2 * d][f][RATE ? pt : 0], sm);
        sm = fma(-lfp, H[2 * d + 1][f][RATE ? pt : 0], sm);
        acc[f] = fma(sc, sm, acc[f]);
      }
    }
  }
  if (node) {
#pragma unroll
    for (int f = 0; f < 5; ++f) R[f * fs + g] = acc[f];
  }
}

// MODE 0: R += viscous rate.  MODE 1: LSERK45 stage in place with the
// inviscid rate R: res = a res + dt (R + viscous), Q = Q + b res.  MODE 2:
// the first stage (a = 0): res = dt (R + viscous) without reading res.  (A
// runtime flag instead of MODE 2 made the compiler duplicate the body and
// hold 200-250 registers.)
template <int N, int MODE>
__global__ void __launch_bounds__(VCfg<N>::NT)
k_visc_apply(DGTables tb, const double* __restrict__ Fv, double* __restrict__ R, double* __restrict__ Q,
             double* __restrict__ res, double a, double b, double dt, DGOrder ord) {
  constexpr int N2 = VCfg<N>::N2, N3 = VCfg<N>::N3, NT = VCfg<N>::NT;
  __shared__ double F[12][N3];
  __shared__ double Tn[6][4][N2];
  // the element of this workgroup in the visiting order (pencils, XCD chunks)
  int e, ne;
  dgdev::block_elements<1>(tb, ord, blockIdx.x, gridDim.x, e, ne);
  const int t = threadIdx.x;
  const int64_t fs = (int64_t)tb.E * N3;
  if constexpr (N3 >= 2) {
    // two nodes per lane and 16-byte load (dword alignment suffices; at odd
    // N^3 the last pair overlaps the one before it)
    constexpr int NP = (N3 + 1) / 2;
    if (t < NP) {
      const int n0 = 2 * t < N3 - 2 ? 2 * t : N3 - 2;
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        double2 w;
        __builtin_memcpy(&w, Fv + c * fs + (int64_t)e * N3 + n0, 16);
        F[c][n0] = w.x;
        F[c][n0 + 1] = w.y;
      }
    }
  } else if (t < N3) {
#pragma unroll
    for (int c = 0; c < 12; ++c) F[c][t] = Fv[c * fs + (int64_t)e * N3 + t];
  }
  const int wave = t >> 6, lane = t & 63;
  using PC = PairCfg<N>;
  if constexpr (!PC::PAIRS) {
    for (int sl = wave; sl < VCfg<N>::NSLOT; sl += VCfg<N>::NW) {
      int face, pt;
      if (face_lane<N>(sl, lane, face, pt)) {
        const int s = face & 1;
        const int en = dgdev::neighbour(tb.nx, tb.ny, tb.nz, e, face >> 1, s ? 1 : -1);
        double acc[4];
        switch (face >> 1) {   // uniform over the wave
          case 0: flux_trace<N, 0>(tb, Fv + (int64_t)en * N3, fs, s, pt, acc); break;
          case 1: flux_trace<N, 1>(tb, Fv + (int64_t)en * N3, fs, s, pt, acc); break;
          default: flux_trace<N, 2>(tb, Fv + (int64_t)en * N3, fs, s, pt, acc); break;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) Tn[face][c][pt] = acc[c];
      }
    }
  } else for (int sl = wave; sl < PC::SLOTS; sl += VCfg<N>::NW) {
    if (sl < PC::WX) {
      // x-faces: one point per lane
      const int it = sl * 64 + lane;
      if (it < 2 * N2) {
        const int s = it >= N2, pt = it - s * N2, face = s;
        const int en = dgdev::neighbour(tb.nx, tb.ny, tb.nz, e, 0, s ? 1 : -1);
        double acc[4];
        flux_trace<N, 0>(tb, Fv + (int64_t)en * N3, fs, s, pt, acc);
#pragma unroll
        for (int c = 0; c < 4; ++c) Tn[face][c][pt] = acc[c];
      }
    } else {
      // y- and z-faces: two points of a row per lane, as in the flux launch
      const int it = (sl - PC::WX) * 64 + lane;
      if (it < PC::NYZ) {
        const int qf = it / (N * PC::H), r = it - qf * (N * PC::H);
        const int b = r / PC::H, c2 = r - b * PC::H;
        const int a0 = 2 * c2 < N - 2 ? 2 * c2 : N - 2;
        const int d = 1 + (qf >> 1), s = qf & 1, face = 2 * d + s;
        const int sm = d == 1 ? N : N2, sb = d == 1 ? N2 : N;
        const int en = dgdev::neighbour(tb.nx, tb.ny, tb.nz, e, d, s ? 1 : -1);
        double acc[2][4];
        flux_trace_pair<N>(tb, Fv + (int64_t)en * N3, fs, s, d, sm, a0 + b * sb, acc);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
          for (int c = 0; c < 4; ++c) Tn[face][c][a0 + h + N * b] = acc[h][c];
        }
      }
    }
  }
  __syncthreads();
  if (t >= N3) return;
  const int i = t % N, j = (t / N) % N, k = t / N2;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int m0, pt;
    line_of<N>(d, i, j, k, m0, pt);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      v[1 + c] += br1_line<N>(tb, F[d * 4 + c], d, m0, pt, Tn[2 * d][c][pt], Tn[2 * d + 1][c][pt]);
  }
  const int64_t g = (int64_t)e * N3 + t;
  if (MODE == 0) {
#pragma unroll
    for (int f = 1; f < 5; ++f) R[f * fs + g] += v[f];
  } else {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      const double rate = R[f * fs + g] + v[f];
      const double r = MODE == 2 ? dt * rate : fma(a, res[f * fs + g], dt * rate);
      res[f * fs + g] = r;
      Q[f * fs + g] = fma(b, r, Q[f * fs + g]);
    }
  }
}

template <int N>
int launch_visc_n(const dg_ctx* c, const double* Q, double* Fv, double* R, double* Qu, double* res, int mode,
                  double a, double b, double dt, int first, bool rate) {
  unsigned grid;
  const DGOrder ord = dg_order(c, 1, &grid);
  const dim3 blk(VCfg<N>::NT);
  if (rate)
    hipLaunchKernelGGL((k_visc_flux<N, true>), dim3(grid), blk, 0, c->stream, c->tab, Q, Fv, R, c->mu, c->kappa, ord);
  else
    hipLaunchKernelGGL((k_visc_flux<N, false>), dim3(grid), blk, 0, c->stream, c->tab, Q, Fv, nullptr, c->mu,
                       c->kappa, ord);
  if (mode == 0)
    hipLaunchKernelGGL((k_visc_apply<N, 0>), dim3(grid), blk, 0, c->stream, c->tab, Fv, R, nullptr, nullptr, a, b,
                       dt, ord);
  else if (first)
    hipLaunchKernelGGL((k_visc_apply<N, 2>), dim3(grid), blk, 0, c->stream, c->tab, Fv, R, Qu, res, a, b, dt, ord);
  else
    hipLaunchKernelGGL((k_visc_apply<N, 1>), dim3(grid), blk, 0, c->stream, c->tab, Fv, R, Qu, res, a, b, dt, ord);
  return (int)hipGetLastError();
}

}  // namespace

int dg_launch_visc(const dg_ctx* c, const double* Q, double* Fv, double* R, double* Qu, double* res, int mode,
                   double a, double b, double dt, int first, bool rate) {
  switch (c->N) {
    case 1: return launch_visc_n<1>(c, Q, Fv, R, Qu, res, mode, a, b, dt, first, rate);
    case 2: return launch_visc_n<2>(c, Q, Fv, R, Qu, res, mode, a, b, dt, first, rate);
    case 3: return launch_visc_n<3>(c, Q, Fv, R, Qu, res, mode, a, b, dt, first, rate);
    case 4: return launch_visc_n<4>(c, Q, Fv, R, Qu, res, mode, a, b, dt, first, rate);
    case 5: return launch_visc_n<5>(c, Q, Fv, R, Qu, res, mode, a, b, dt, first, rate);
    case 6: return launch_visc_n<6>(c, Q, Fv, R, Qu, res, mode, a, b, dt, first, rate);
    case 7: return launch_visc_n<7>(c, Q, Fv, R, Qu, res, mode, a, b, dt, first, rate);
    case 8: return launch_visc_n<8>(c, Q, Fv, R, Qu, res, mode, a, b, dt, first, rate);
    default: return (int)hipErrorInvalidValue;
  }
}
