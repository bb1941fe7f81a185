// Kinetic-energy-preserving split-form volume term (flux differencing with
// the Kennedy-Gruber two-point flux) on the collocated Gauss-Legendre basis.
//
// The paper cites kinetic-energy-preserving flux schemes of its authors' DG
// framework (reference list) without printing one; the reading taken:
//   two-point flux in direction d, {a} the mean of two states' values,
//   e = E / rho:  {rho}{u_d},  {rho}{u_d}{u_k} + {p} delta_kd,
//                 {rho}{u_d}{e} + {p}{u_d};
//   the Gauss-Legendre nodes do not include the element ends, so each d-line
//   couples its N nodes with the two face traces through the hybridised
//   summation-by-parts operator; written out per node i of the line (mass
//   matrix divided out, D_ia = l_a'(xi_i), l(+-1) the face interpolation
//   weights):
//     dQ_i/dt -= (2/h_d) [ sum_a 2 D_ia f_S(Q_i, Q_a)
//                 + l_i(+1)/w_i B_+ - l_i(-1)/w_i B_- ],
//     B_f = f_S(Q_i, Q~_f) - sum_a l_a(f) f_S(Q_i, Q_a)
//           + F*_f - sum_a l_a(f) f_S(Q~_f, Q_a),
//   Q~_f the element's own trace on face f, F*_f the local Lax-Friedrichs
//   flux of the standard scheme there.  With the central two-point flux this
//   is exactly the standard weak form.
//
// One workgroup per element (elements visited in the neighbour-read stage's
// order: pencils, each XCD a contiguous part), one thread per node (the
// pairwise fluxes make the volume term O(N^4) per element); the face points
// of each direction on waves of their own.  The last two terms of B_f depend on
// the face point only, not on the node along the line: they are formed once
// per face point in the face phase, so a node evaluates N + 2 two-point
// fluxes per direction and each face point N (3N + 6 per node and 6 per
// node for the faces, against 9N + 6 when every node forms all of B_f).
// MODE 0: R = dQ/dt.  MODE 1: LSERK45 stage, Qout = Qin + b res
// with res = a res + dt R in place (Qin and Qout differ: neighbours read
// Qin).  MODE 2: the first stage (res = dt R without reading res).

#include "dg_internal.h"
#include "stage_fp64.h"
#include "stage_nb.h"

namespace {

template <int N>
struct SCfg {
  static constexpr int N2 = N * N;
  static constexpr int N3 = N * N * N;
  // N >= 5: the face points of one direction (both sides) on WPD waves of
  // their own, so that the direction is uniform over a wave; below, where a
  // direction's points fill at most half a wave, the 6 N^2 points in order
  // (separate waves would add waves that idle in the volume phase)
  static constexpr bool WAVES = 2 * N2 > 32;
  static constexpr int WPD = (2 * N2 + 63) / 64;
  // whole waves covering the nodes and the face phase in one round (a wave
  // that took two directions one after the other would hold both variants'
  // registers, and spilled)
  static constexpr int NF = WAVES ? 3 * WPD * 64 : 6 * N2;
  static constexpr int NT = ((N3 > NF ? N3 : NF) + 63) / 64 * 64;
  // the element's state in LDS for its own face traces (at N = 8 the 20 KB
  // would leave one workgroup per CU: there the traces read global memory)
  static constexpr bool QL = N < 8;
  static constexpr int NQ = QL ? N3 : 1;
  // the neighbour's face traces formed while the node primitives are staged
  // (their loads overlap the staging), and the update's state taken from
  // LDS; at N = 7 either costs registers (the update 150 -> 168 VGPRs, the
  // early traces spills) and time, so there the traces follow the staging
  // and the update reads global memory
  static constexpr bool EARLY = N != 7;
  // the line weights folded into the two-point flux (kg_acc) up to N = 5;
  // from N = 6 the flux is formed and then accumulated (the folded form ran
  // slower there: p = 5 by a third, p = 6 by 7%, p = 7 even)
  static constexpr bool FOLD = N <= 5;
};

// Half the primitives of a state: rho, u, v, w, p, e = E / rho, each times
// 1/2, so that the mean of two states' values is one addition (halving is
// exact, so a/2 + b/2 is (a + b)/2 bit for bit).
struct Prim {
  double r, u[3], p, e;
};

__device__ __forceinline__ Prim to_prim(const double* q, double gm1) {
  Prim s;
  const double ri = dgdev::recip(q[0]);
  s.r = 0.5 * q[0];
  s.u[0] = 0.5 * (q[1] * ri);
  s.u[1] = 0.5 * (q[2] * ri);
  s.u[2] = 0.5 * (q[3] * ri);
  s.p = 0.5 * (gm1 * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) * ri));
  s.e = 0.5 * (q[4] * ri);
  return s;
}

// Kennedy-Gruber two-point flux in direction D of two states given by their
// half primitives.
template <int D>
__device__ __forceinline__ void kg_flux(const Prim& a, const Prim& b, double* f) {
  const double rho = a.r + b.r;
  const double ud = a.u[D] + b.u[D];
  const double pm = a.p + b.p;
  const double mass = rho * ud;
  f[0] = mass;
#pragma unroll
  for (int k = 0; k < 3; ++k) f[1 + k] = mass * (a.u[k] + b.u[k]);
  f[1 + D] += pm;
  f[4] = mass * (a.e + b.e) + pm * ud;
}

// The same, accumulated with weight c: the weight enters the mass
// flux and the mean pressure once (c {rho}{u_d} and c {p}), which then scale
// the means (16 operations per pair, against 13 for the flux and 5 for a
// separate accumulation).
template <int D>
__device__ __forceinline__ void kg_acc(const Prim& a, const Prim& b, double c, double* acc) {
  const double rho = a.r + b.r;
  double um[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) um[k] = a.u[k] + b.u[k];
  const double cm = c * (rho * um[D]);
  const double cp = c * (a.p + b.p);
  acc[0] += cm;
#pragma unroll
  for (int k = 0; k < 3; ++k) acc[1 + k] = fma(cm, um[k], acc[1 + k]);
  acc[1 + D] += cp;
  acc[4] = fma(cm, a.e + b.e, acc[4]);
  acc[4] = fma(cp, um[D], acc[4]);
}

// kg_acc as the flux first, then five multiply-adds (the form used from
// N = 6), or folded.
template <int N, int D>
__device__ __forceinline__ void kg_acc_n(const Prim& a, const Prim& b, double c, double* acc) {
  if constexpr (SCfg<N>::FOLD) {
    kg_acc<D>(a, b, c, acc);
  } else {
    double f[5];
    kg_flux<D>(a, b, f);
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[v] = fma(c, f[v], acc[v]);
  }
}

// A state's primitives in LDS: six doubles at a 16-byte aligned place, read
// and written as three 16-byte accesses.
__device__ __forceinline__ Prim lds_prim(const double* p) {
  const double2* q = reinterpret_cast<const double2*>(p);
  const double2 a = q[0], b = q[1], c = q[2];
  Prim s;
  s.r = a.x;
  s.u[0] = a.y;
  s.u[1] = b.x;
  s.u[2] = b.y;
  s.p = c.x;
  s.e = c.y;
  return s;
}

__device__ __forceinline__ void lds_put(double* p, const Prim& s) {
  double2* q = reinterpret_cast<double2*>(p);
  q[0] = make_double2(s.r, s.u[0]);
  q[1] = make_double2(s.u[1], s.u[2]);
  q[2] = make_double2(s.p, s.e);
}

// Volume and face terms of direction D for node (m0 along the line, pt
// across it) of the element whose node primitives are P, accumulated (with
// the -(2/h_D) factor) into out.  The two face terms' sums over the line
// enter linearly, so they fold into the volume weights:
//   W_ia = 2 D_ia - l_i(+1)/w_i l_a(+1) + l_i(-1)/w_i l_a(-1),
//   rate_i = sum_a W_ia f_S(Q_i, Q_a) + l_i(+1)/w_i (f_S(Q_i, Q~_+) + G_+)
//            - l_i(-1)/w_i (f_S(Q_i, Q~_-) + G_-),
// G holding, per face point, the part of the face term that does not depend
// on the node along the line: F*_f - sum_a l_a(f) f_S(Q~_f, Q_a).
template <int N, int D>
__device__ __forceinline__ void split_line(const DGTables& tb, const double (*P)[6], const double (*Wm)[N],
                                           const double (*Tp)[SCfg<N>::N2][6], const double (*G)[SCfg<N>::N2][6],
                                           int m0, int pt, double* out) {
  const Prim si = lds_prim(P[dgdev::tnode<N>(D, m0, pt)]);
  const double sc = tb.sc[D];
  if constexpr (SCfg<N>::FOLD) {
    // sum_a W_ia f_S(Q_i, Q_a) + l_i(+1)/w_i (f_S(Q_i, Q~_+) + G_+)
    //   - l_i(-1)/w_i (f_S(Q_i, Q~_-) + G_-), each flux with its weight
    const double lp = tb.liftp[m0], lm = tb.liftm[m0];
    double vol[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) vol[v] = fma(lp, G[2 * D + 1][pt][v], -lm * G[2 * D][pt][v]);
#pragma unroll
    for (int a = 0; a < N; ++a) kg_acc<D>(si, lds_prim(P[dgdev::tnode<N>(D, a, pt)]), Wm[m0][a], vol);
    kg_acc<D>(si, lds_prim(Tp[2 * D][pt]), -lm, vol);
    kg_acc<D>(si, lds_prim(Tp[2 * D + 1][pt]), lp, vol);
#pragma unroll
    for (int v = 0; v < 5; ++v) out[v] = fma(-sc, vol[v], out[v]);
  } else {
    double vol[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // sum_a W_ia f_S(Q_i, Q_a)
#pragma unroll
    for (int a = 0; a < N; ++a) {
      const Prim sa = lds_prim(P[dgdev::tnode<N>(D, a, pt)]);
      double f[5];
      kg_flux<D>(si, sa, f);
      const double w = Wm[m0][a];
#pragma unroll
      for (int v = 0; v < 5; ++v) vol[v] = fma(w, f[v], vol[v]);
    }
    double br[2][5];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const Prim tf = lds_prim(Tp[2 * D + s][pt]);
      double fi[5];
      kg_flux<D>(si, tf, fi);                      // f_S(Q_i, Q~_f)
#pragma unroll
      for (int v = 0; v < 5; ++v) br[s][v] = fi[v] + G[2 * D + s][pt][v];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v)
      out[v] -= sc * (vol[v] + tb.liftp[m0] * br[1][v] - tb.liftm[m0] * br[0][v]);
  }
}

// sum_a l_a(f) f_S(Q~_f, Q_a) along the D-line through face point pt
// (weights c = l(-1) or l(+1) of the face's side).
template <int N, int D>
__device__ __forceinline__ void face_line_sum(const double (*P)[6], const Prim& tf, const double* c,
                                              int pt, double* sf) {
#pragma unroll
  for (int a = 0; a < N; ++a) {
    const Prim sa = lds_prim(P[dgdev::tnode<N>(D, a, pt)]);
    kg_acc_n<N, D>(tf, sa, c[a], sf);
  }
}

// The neighbour's trace at face point i (side s = i / N^2, point pt) of
// direction D, interpolated along its normal line from global memory (no
// shared memory: issued before the node primitives are staged).
template <int N, int D>
__device__ __forceinline__ void nbr_trace(const DGTables& tb, const double* __restrict__ Qin, int64_t fs, int e,
                                          int i, double* nbr) {
  constexpr int N2 = SCfg<N>::N2, N3 = SCfg<N>::N3;
  const int s = i / N2, pt = i - s * N2;
  const int en = dgdev::neighbour(tb.nx, tb.ny, tb.nz, e, D, s ? 1 : -1);
  const double* qn = Qin + (int64_t)en * N3;
#pragma unroll
  for (int f = 0; f < 5; ++f) nbr[f] = 0.0;
#pragma unroll
  for (int m = 0; m < N; ++m) {
    const int node = dgdev::tnode<N>(D, m, pt);
    const double wn = s ? tb.lm[m] : tb.lp[m];   // the neighbour's trace on its opposite face
#pragma unroll
    for (int f = 0; f < 5; ++f) nbr[f] = fma(wn, qn[f * fs + node], nbr[f]);
  }
}

// Face point i of direction D: the element's own trace (from its state in
// LDS; from global memory at N = 8), the neighbour's (given, or with EARLY
// off interpolated here beside the own trace), the Lax-Friedrichs flux, and
// into LDS the point's G term and its own trace's primitives.  The side is a
// per-lane select, so lanes of both sides of a direction run the same
// instructions.
template <int N, int D>
__device__ __forceinline__ void split_face(const DGTables& tb, const double* __restrict__ Qin, int64_t fs, int e,
                                           int i, const double* nbr_in, const double (*Qs)[SCfg<N>::NQ],
                                           const double (*P)[6], double (*Tp)[SCfg<N>::N2][6],
                                           double (*G)[SCfg<N>::N2][6]) {
  constexpr int N2 = SCfg<N>::N2, N3 = SCfg<N>::N3;
  constexpr bool EARLY = SCfg<N>::EARLY;
  const int s = i / N2, pt = i - s * N2;
  const int face = 2 * D + s;
  const double* qe = Qin + (int64_t)e * N3;
  const double* qn = Qin + (int64_t)(EARLY ? 0 : dgdev::neighbour(tb.nx, tb.ny, tb.nz, e, D, s ? 1 : -1)) * N3;
  double own[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, nbr[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) nbr[f] = EARLY ? nbr_in[f] : 0.0;
#pragma unroll
  for (int m = 0; m < N; ++m) {
    const int node = dgdev::tnode<N>(D, m, pt);
    const double wo = s ? tb.lp[m] : tb.lm[m];   // own trace on this face
    const double wn = s ? tb.lm[m] : tb.lp[m];   // the neighbour's trace on its opposite face
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      own[f] = fma(wo, SCfg<N>::QL ? Qs[f][SCfg<N>::QL ? node : 0] : qe[f * fs + node], own[f]);
      if (!EARLY) nbr[f] = fma(wn, qn[f * fs + node], nbr[f]);
    }
  }
  // the face's -d side state first
  double mn[5], pl[5], fl[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    mn[f] = s ? own[f] : nbr[f];
    pl[f] = s ? nbr[f] : own[f];
  }
  dgdev::lf_flux_d<D>(mn, pl, tb.gamma, tb.gm1, fl);
  const Prim so = to_prim(own, tb.gm1);
  double c[N], sf[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < N; ++a) c[a] = s ? tb.lp[a] : tb.lm[a];
  face_line_sum<N, D>(P, so, c, pt, sf);
#pragma unroll
  for (int f = 0; f < 5; ++f) G[face][pt][f] = fl[f] - sf[f];
  lds_put(Tp[face][pt], so);
}

template <int N, int MODE>
__global__ void __launch_bounds__(SCfg<N>::NT) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_split(DGTables tb, const double* __restrict__ Qin, double* __restrict__ Qout, double* __restrict__ RR, double a,
        double b, double dt, DGOrder ord) {
  constexpr int N2 = SCfg<N>::N2, N3 = SCfg<N>::N3, WPD = SCfg<N>::WPD;
  // per node / face point six doubles (16-byte aligned: three 16-byte accesses)
  __shared__ __align__(16) double P[N3][6];        // node primitives
  __shared__ __align__(16) double Tp[6][N2][6];    // own trace primitives per face (2d + side)
  __shared__ __align__(16) double G[6][N2][6];     // per face point: Lax-Friedrichs flux - sum_a l_a f_S(Q~_f, Q_a)
  __shared__ double Qs[5][SCfg<N>::NQ];             // the element's state (its own face traces)
  __shared__ double Wm[N][N];        // W_ia = 2 D_ia - l_i(1) l_a(1) / w_i + l_i(-1) l_a(-1) / w_i
  // the element of this workgroup in the visiting order (pencils, XCD chunks)
  int e, ne;
  dgdev::block_elements<1>(tb, ord, blockIdx.x, gridDim.x, e, ne);
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  const int64_t fs = (int64_t)tb.E * N3;
  const double* qe = Qin + (int64_t)e * N3;
  if (t < N2) {
    const int i = t / N, aa = t % N;
    // Dh[a N + i] = w_i l_a'(xi_i) / w_a
    const double dia = tb.Dh[aa * N + i] * tb.w[aa] / tb.w[i];   // D_ia = l_a'(xi_i)
    Wm[i][aa] = 2.0 * dia - tb.liftp[i] * tb.lp[aa] + tb.liftm[i] * tb.lm[aa];
  }
  // face points: wave w < 3 WPD takes 64 points of direction w / WPD (or,
  // below N = 5, thread t takes point t); the neighbour's trace needs no
  // shared memory, so its loads can be issued with the element's own
  const int d = SCfg<N>::WAVES ? wave / WPD : t / (2 * N2);
  const int fi = SCfg<N>::WAVES ? (wave - d * WPD) * 64 + lane : t - d * 2 * N2;
  const bool fpt = d < 3 && fi < 2 * N2;
  double q[5], nbr[5];
  if (t < N3) {
#pragma unroll
    for (int f = 0; f < 5; ++f) q[f] = qe[f * fs + t];
  }
  if (SCfg<N>::EARLY && fpt) {
    if (d == 0) nbr_trace<N, 0>(tb, Qin, fs, e, fi, nbr);
    else if (d == 1) nbr_trace<N, 1>(tb, Qin, fs, e, fi, nbr);
    else nbr_trace<N, 2>(tb, Qin, fs, e, fi, nbr);
  }
  if (t < N3) {
    if (SCfg<N>::QL) {
#pragma unroll
      for (int f = 0; f < 5; ++f) Qs[f][SCfg<N>::QL ? t : 0] = q[f];
    }
    const Prim s = to_prim(q, tb.gm1);
    lds_put(P[t], s);
  }
  __syncthreads();   // the face phase reads the node primitives
  if (fpt) {
    if (d == 0) split_face<N, 0>(tb, Qin, fs, e, fi, nbr, Qs, P, Tp, G);
    else if (d == 1) split_face<N, 1>(tb, Qin, fs, e, fi, nbr, Qs, P, Tp, G);
    else split_face<N, 2>(tb, Qin, fs, e, fi, nbr, Qs, P, Tp, G);
  }
  __syncthreads();
  if (t >= N3) return;
  const int i = t % N, j = (t / N) % N, k = t / N2;
  double rate[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  split_line<N, 0>(tb, P, Wm, Tp, G, i, j + N * k, rate);
  split_line<N, 1>(tb, P, Wm, Tp, G, j, i + N * k, rate);
  split_line<N, 2>(tb, P, Wm, Tp, G, k, i + N * j, rate);
  const int64_t g = (int64_t)e * N3 + t;
  if (MODE == 0) {
#pragma unroll
    for (int f = 0; f < 5; ++f) RR[f * fs + g] = rate[f];
  } else {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      const double r = MODE == 2 ? dt * rate[f] : fma(a, RR[f * fs + g], dt * rate[f]);
      RR[f * fs + g] = r;
      Qout[f * fs + g] = fma(b, r, SCfg<N>::QL && SCfg<N>::EARLY ? Qs[f][SCfg<N>::QL ? t : 0] : Qin[f * fs + g]);
    }
  }
}

template <int N>
int launch_split_n(const dg_ctx* c, const double* Qin, double* Qout, double* RR, int mode, double a, double b,
                   double dt) {
  unsigned grid;
  const DGOrder ord = dg_order(c, 1, &grid);
  const dim3 blk(SCfg<N>::NT);
  if (mode == 0)
    hipLaunchKernelGGL((k_split<N, 0>), dim3(grid), blk, 0, c->stream, c->tab, Qin, Qout, RR, a, b, dt, ord);
  else if (mode == 2)
    hipLaunchKernelGGL((k_split<N, 2>), dim3(grid), blk, 0, c->stream, c->tab, Qin, Qout, RR, a, b, dt, ord);
  else
    hipLaunchKernelGGL((k_split<N, 1>), dim3(grid), blk, 0, c->stream, c->tab, Qin, Qout, RR, a, b, dt, ord);
  return (int)hipGetLastError();
}

}  // namespace

int dg_launch_split(const dg_ctx* c, const double* Qin, double* Qout, double* RR, int mode, double a, double b,
                    double dt) {
  switch (c->N) {
    case 1: return launch_split_n<1>(c, Qin, Qout, RR, mode, a, b, dt);
    case 2: return launch_split_n<2>(c, Qin, Qout, RR, mode, a, b, dt);
    case 3: return launch_split_n<3>(c, Qin, Qout, RR, mode, a, b, dt);
    case 4: return launch_split_n<4>(c, Qin, Qout, RR, mode, a, b, dt);
    case 5: return launch_split_n<5>(c, Qin, Qout, RR, mode, a, b, dt);
    case 6: return launch_split_n<6>(c, Qin, Qout, RR, mode, a, b, dt);
    case 7: return launch_split_n<7>(c, Qin, Qout, RR, mode, a, b, dt);
    case 8: return launch_split_n<8>(c, Qin, Qout, RR, mode, a, b, dt);
    default: return (int)hipErrorInvalidValue;
  }
}
