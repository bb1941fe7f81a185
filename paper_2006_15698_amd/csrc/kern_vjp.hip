// Adjoint (vector-Jacobian product) of the DG Euler right-hand side for
// gfx950: gQ = (dR/dQ)^T gR, FP64.
//
// R of Eq. (5), per element e and node s with normal index m and
// tangential point pt along direction d:
//   R_s = sum_d (2/h_d) [ sum_a Dh[m][a] F^d(Q_line(a))
//                         + liftm[m] F*_{-d}(pt) - liftp[m] F*_{+d}(pt) ]
//   F*_{+d} = LF(T_{e,+d}, T_{e+d,-d}),  T_{e,+-d}(pt) = sum_m l_m(+-1) Q_e(line)
// Reverse mode, per element (no atomics: each side of a face computes the
// adjoint of its own trace):
//   1. lifted adjoint traces G_{e,+-d}(pt) = sum_m lift+-[m] gR_e(line) and
//      forward traces T of Q, of this element and of its neighbours (read
//      from the neighbours' Q and gR in the same launch by k_vjp_nb, or
//      exchanged through trace buffers by k_vtrace + k_vjp);
//   2. face flux adjoint gF*_{face} = (2/h_d)(G_{plus elem,-d} - G_{minus elem,+d}),
//      then the LF Jacobian transpose for this element's side, then the
//      trace transpose l_m(+-1) back onto the line;
//   3. volume: gF^d(t) = (2/h_d) sum_i Dh[i][m_t] gR(line i) (transposed
//      contraction) and the 5x5 flux Jacobian transpose at node t.
// Branch conventions at the kinks: |x|' = +1 for x >= 0, and the wave speed
// max(l-, l+) differentiates the - side when l- >= l+ (the forward's choice).

#include "dg_internal.h"
#include "stage_nb.h"

namespace {

template <int N> struct VCfg;
template <> struct VCfg<1> { static constexpr int EPB = 64; static constexpr int NT = 64; };
template <> struct VCfg<2> { static constexpr int EPB = 16; static constexpr int NT = 128; };
template <> struct VCfg<3> { static constexpr int EPB = 9; static constexpr int NT = 256; };
template <> struct VCfg<4> { static constexpr int EPB = 4; static constexpr int NT = 256; };
template <> struct VCfg<5> { static constexpr int EPB = 2; static constexpr int NT = 256; };
template <> struct VCfg<6> { static constexpr int EPB = 1; static constexpr int NT = 256; };
template <> struct VCfg<7> { static constexpr int EPB = 1; static constexpr int NT = 384; };
template <> struct VCfg<8> { static constexpr int EPB = 1; static constexpr int NT = 512; };

template <int N>
__device__ __forceinline__ int vnode(int d, int m, int pt) {
  if (d == 0) return pt * N + m;
  if (d == 1) return (pt / N) * N * N + m * N + (pt % N);
  return m * N * N + pt;
}

__device__ __forceinline__ int vneighbour(const DGTables& tb, int e, int d, int dir) {
  const int nx = tb.nx, ny = tb.ny, nz = tb.nz;
  const int ex = e % nx;
  const int r = e / nx;
  const int ey = r % ny;
  const int ez = r / ny;
  if (d == 0) {
    int x = ex + dir;
    x = x < 0 ? nx - 1 : (x >= nx ? 0 : x);
    return e + (x - ex);
  }
  if (d == 1) {
    int y = ey + dir;
    y = y < 0 ? ny - 1 : (y >= ny ? 0 : y);
    return e + (y - ey) * nx;
  }
  int z = ez + dir;
  z = z < 0 ? nz - 1 : (z >= nz ? 0 : z);
  return e + (z - ez) * nx * ny;
}

// out += (dF^d/dQ)^T g at state q (Eq. (2) with the pressure of Eq. (3)).
template <int d>
__device__ __forceinline__ void flux_vjp(const double* q, const double* g, double gm1, double* out) {
  const double r = dgdev::recip(q[0]);
  const double u0 = q[1] * r, u1 = q[2] * r, u2 = q[3] * r;
  const double ud = d == 0 ? u0 : (d == 1 ? u1 : u2);
  const double pr = gm1 * (q[4] - 0.5 * (q[1] * u0 + q[2] * u1 + q[3] * u2));
  const double gd = d == 0 ? g[1] : (d == 1 ? g[2] : g[3]);
  // S = g0 m_d + sum_k g_k m_k u_d + g_d p + g4 (E + p) u_d
  const double B = g[1] * q[1] + g[2] * q[2] + g[3] * q[3] + g[4] * (q[4] + pr);  // dS/du_d
  const double P = gd + g[4] * ud;                                                // dS/dp
  const double usq = u0 * u0 + u1 * u1 + u2 * u2;
  out[0] += -B * ud * r + P * gm1 * 0.5 * usq;
  out[1] += g[1] * ud - P * gm1 * u0 + (d == 0 ? g[0] + B * r : 0.0);
  out[2] += g[2] * ud - P * gm1 * u1 + (d == 1 ? g[0] + B * r : 0.0);
  out[3] += g[3] * ud - P * gm1 * u2 + (d == 2 ? g[0] + B * r : 0.0);
  out[4] += g[4] * ud + P * gm1;
}

// Local wave speed l = |u_d| + c and its gradient dl/dq.
template <int d>
__device__ __forceinline__ double wave_speed_grad(const double* q, double gamma, double gm1, double* dl) {
  const double r = dgdev::recip(q[0]);
  const double u0 = q[1] * r, u1 = q[2] * r, u2 = q[3] * r;
  const double ud = d == 0 ? u0 : (d == 1 ? u1 : u2);
  const double usq = u0 * u0 + u1 * u1 + u2 * u2;
  const double e = gm1 * (q[4] * r - 0.5 * usq);  // p / rho
  const double c = dgdev::root(gamma * e);
  const double sg = ud >= 0.0 ? 1.0 : -1.0;
  const double k = gamma * dgdev::recip(2.0 * c);
  // de/drho = gm1 (-E/rho + |u|^2)/rho, de/dm_k = -gm1 u_k / rho, de/dE = gm1 / rho
  dl[0] = sg * (-ud * r) + k * gm1 * (-q[4] * r + usq) * r;
  dl[1] = (d == 0 ? sg * r : 0.0) - k * gm1 * u0 * r;
  dl[2] = (d == 1 ? sg * r : 0.0) - k * gm1 * u1 * r;
  dl[3] = (d == 2 ? sg * r : 0.0) - k * gm1 * u2 * r;
  dl[4] = k * gm1 * r;
  return fabs(ud) + c;
}

// Transpose of the local Lax-Friedrichs Jacobian for one side, applied to g:
// minus side:  (1/2) A(qm)^T g + (lambda/2) g - (1/2)(g . (qp - qm)) dlambda/dqm
// plus side:   (1/2) A(qp)^T g - (lambda/2) g - (1/2)(g . (qp - qm)) dlambda/dqp
template <int d>
__device__ __forceinline__ void lf_vjp_d(const double* qm, const double* qp, double gamma, double gm1,
                                         const double* g, bool minus_side, double* out) {
  double dlm[5], dlp[5];
  const double lm = wave_speed_grad<d>(qm, gamma, gm1, dlm);
  const double lp = wave_speed_grad<d>(qp, gamma, gm1, dlp);
  const bool pick_m = lm >= lp;
  const double lam = pick_m ? lm : lp;
  double gdel = 0.0;
#pragma unroll
  for (int f = 0; f < 5; ++f) gdel += g[f] * (qp[f] - qm[f]);
  double hg[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    hg[f] = 0.5 * g[f];
    out[f] = 0.0;
  }
  double qs[5], dl[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    qs[f] = minus_side ? qm[f] : qp[f];
    dl[f] = minus_side ? dlm[f] : dlp[f];
  }
  flux_vjp<d>(qs, hg, gm1, out);
  const bool own_selected = minus_side ? pick_m : !pick_m;
  const double sl = minus_side ? 0.5 * lam : -0.5 * lam;
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    out[f] += sl * g[f];
    if (own_selected) out[f] -= 0.5 * gdel * dl[f];
  }
}

__device__ __forceinline__ void lf_vjp(const double* qm, const double* qp, int d, double gamma, double gm1,
                                       const double* g, bool minus_side, double* out) {
  if (d == 0) lf_vjp_d<0>(qm, qp, gamma, gm1, g, minus_side, out);
  else if (d == 1) lf_vjp_d<1>(qm, qp, gamma, gm1, g, minus_side, out);
  else lf_vjp_d<2>(qm, qp, gamma, gm1, g, minus_side, out);
}

template <int N>
__device__ __forceinline__ double line_sum(const double* s, const double* coef, int d, int pt) {
  double v = 0.0;
#pragma unroll
  for (int m = 0; m < N; ++m) v = fma(coef[m], s[vnode<N>(d, m, pt)], v);
  return v;
}

// Face traces of a state (coefficients l(+-1)) or lifted traces of an
// adjoint (coefficients l(+-1)/w), all six faces, same layout as the
// forward traces: T[(face*5+f)][e][pt].
template <int N, bool LIFT>
__global__ void __launch_bounds__(VCfg<N>::NT)
k_vtrace(DGTables tb, const double* __restrict__ X, double* __restrict__ T) {
  constexpr int EPB = VCfg<N>::EPB, NT = VCfg<N>::NT;
  constexpr int N2 = N * N, N3 = N2 * N, NODES = EPB * N3, FP = EPB * N2;
  __shared__ double sX[DG_NF][NODES];
  __shared__ double sCm[N], sCp[N];
  const int tid = threadIdx.x;
  const int e0 = blockIdx.x * EPB;
  const int E = tb.E;
  const int64_t EN3 = (int64_t)E * N3, EN2 = (int64_t)E * N2;
  if (tid < N) {
    sCm[tid] = LIFT ? tb.liftm[tid] : tb.lm[tid];
    sCp[tid] = LIFT ? tb.liftp[tid] : tb.lp[tid];
  }
  for (int x = tid; x < NODES; x += NT) {
    if (e0 + x / N3 < E) {
#pragma unroll
      for (int f = 0; f < 5; ++f) sX[f][x] = X[f * EN3 + (int64_t)e0 * N3 + x];
    }
  }
  __syncthreads();
  for (int it = tid; it < 30 * FP; it += NT) {
    const int pt = it % N2;
    const int r1 = it / N2;
    const int fel = r1 % EPB;
    const int r2 = r1 / EPB;
    const int f = r2 % 5;
    const int face = r2 / 5;
    const int ee = e0 + fel;
    if (ee >= E) continue;
    const double* coef = (face & 1) ? sCp : sCm;
    T[(int64_t)(face * 5 + f) * EN2 + (int64_t)ee * N2 + pt] = line_sum<N>(&sX[f][fel * N3], coef, face >> 1, pt);
  }
}

template <int N>
__global__ void __launch_bounds__(VCfg<N>::NT)
k_vjp(DGTables tb, const double* __restrict__ Q, const double* __restrict__ gR, const double* __restrict__ TQ,
      const double* __restrict__ TG, double* __restrict__ gQ) {
  constexpr int EPB = VCfg<N>::EPB, NT = VCfg<N>::NT;
  constexpr int N2 = N * N, N3 = N2 * N, NODES = EPB * N3, FP = EPB * N2;
  constexpr int NITEM = 6 * FP;
  __shared__ double sQ[DG_NF][NODES];
  __shared__ double sG[DG_NF][NODES];
  __shared__ double sH[6][DG_NF][FP];
  __shared__ double sDh[N * N];
  __shared__ double sLm[N], sLp[N], sLiftm[N], sLiftp[N];

  const int tid = threadIdx.x;
  const int E = tb.E;
  const int64_t EN3 = (int64_t)E * N3, EN2 = (int64_t)E * N2;
  const int e0 = blockIdx.x * EPB;
  for (int x = tid; x < N * N; x += NT) sDh[x] = tb.Dh[x];
  if (tid < N) {
    sLm[tid] = tb.lm[tid];
    sLp[tid] = tb.lp[tid];
    sLiftm[tid] = tb.liftm[tid];
    sLiftp[tid] = tb.liftp[tid];
  }
  const bool nthr = tid < NODES;
  const int el = tid / N3;
  const int t = tid - el * N3;
  const int ni = t % N, nj = (t / N) % N, nk = t / N2;
  const int e = e0 + el;
  const bool act = nthr && e < E;
  const int64_t gofs = (int64_t)e * N3 + t;
  double q[5], g[5];
  if (act) {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      q[f] = Q[f * EN3 + gofs];
      g[f] = gR[f * EN3 + gofs];
    }
  } else {
    q[0] = 1.0; q[1] = 0.0; q[2] = 0.0; q[3] = 0.0; q[4] = 2.5;
#pragma unroll
    for (int f = 0; f < 5; ++f) g[f] = 0.0;
  }
  if (nthr) {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      sQ[f][tid] = q[f];
      sG[f][tid] = g[f];
    }
  }
  __syncthreads();

  // ---- face items: adjoint of this element's side of every face
  for (int it = tid; it < NITEM; it += NT) {
    const int face = it / FP;
    const int rem = it - face * FP;
    const int fel = rem / N2;
    const int pt = rem - fel * N2;
    const int ee = e0 + fel;
    const int d = face >> 1, side = face & 1;
    double qo[5], go[5], qn[5], gn[5], gq[5];
    if (ee < E) {
      const int nbe = vneighbour(tb, ee, d, side ? 1 : -1);
      const int oface = 2 * d + (1 - side);
      const double* coefq = side ? sLp : sLm;
      const double* coefg = side ? sLiftp : sLiftm;
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        qo[f] = line_sum<N>(&sQ[f][fel * N3], coefq, d, pt);
        go[f] = line_sum<N>(&sG[f][fel * N3], coefg, d, pt);
        qn[f] = TQ[(int64_t)(oface * 5 + f) * EN2 + (int64_t)nbe * N2 + pt];
        gn[f] = TG[(int64_t)(oface * 5 + f) * EN2 + (int64_t)nbe * N2 + pt];
      }
      const double sc = tb.sc[d];
      double gf[5];
      // + face: this element is the minus side, the neighbour the plus side.
#pragma unroll
      for (int f = 0; f < 5; ++f) gf[f] = side ? sc * (gn[f] - go[f]) : sc * (go[f] - gn[f]);
      double qm[5], qp[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        qm[f] = side ? qo[f] : qn[f];
        qp[f] = side ? qn[f] : qo[f];
      }
      lf_vjp(qm, qp, d, tb.gamma, tb.gm1, gf, side != 0, gq);
    } else {
#pragma unroll
      for (int f = 0; f < 5; ++f) gq[f] = 0.0;
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) sH[face][f][fel * N2 + pt] = gq[f];
  }
  __syncthreads();

  if (!act) return;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int m = d == 0 ? ni : (d == 1 ? nj : nk);
    const int pt = d == 0 ? nj + N * nk : (d == 1 ? ni + N * nk : ni + N * nj);
    const double sc = tb.sc[d];
    double gF[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < N; ++i) s = fma(sDh[i * N + m], sG[f][el * N3 + vnode<N>(d, i, pt)], s);
      gF[f] = sc * s;
    }
    if (d == 0) flux_vjp<0>(q, gF, tb.gm1, acc);   // d is constant after unrolling
    else if (d == 1) flux_vjp<1>(q, gF, tb.gm1, acc);
    else flux_vjp<2>(q, gF, tb.gm1, acc);
#pragma unroll
    for (int f = 0; f < 5; ++f)
      acc[f] += sLp[m] * sH[2 * d + 1][f][el * N2 + pt] + sLm[m] * sH[2 * d][f][el * N2 + pt];
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) gQ[f * EN3 + gofs] = acc[f];
}

// Neighbour-read adjoint: one launch, no trace buffers (the exchange of
// the forward neighbour-read stage, stage_nb.h).  A workgroup owns EPB
// consecutive elements of one x-row; the state Q and the adjoint gR of the
// block and of its left and right x-neighbours are staged in LDS, the y/z
// neighbours' traces of Q (l(-+1)) and lifted traces of gR (lift(-+1)) are
// read by waves that each handle one face.  Same arithmetic as k_vtrace +
// k_vjp (same FMA chains for every trace), so the results are bitwise equal.
template <int N, int EPB>
struct VjpSmem {
  static constexpr int N3 = N * N * N;
  static constexpr int NH = (EPB + 2) * N3;
  static constexpr int FP = EPB * N * N;
  static constexpr int size = 10 * NH + 30 * FP + N * N + 4 * N;
};

// Q trace (coefficients cq) and lifted gR trace (coefficients cg) of the
// neighbour chunk element fel at point pt of our face (D, SIDE).
template <int N, int D>
__device__ __forceinline__ void chunk_trace2(const double* __restrict__ Q, const double* __restrict__ G, int64_t EN3,
                                             int64_t cofs, int pt, const double* cq, const double* cg, double* qn,
                                             double* gn) {
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const double* qf = Q + f * EN3 + cofs;
    const double* gf = G + f * EN3 + cofs;
    double vq = 0.0, vg = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      vq = fma(cq[m], qf[vnode<N>(D, m, pt)], vq);
      vg = fma(cg[m], gf[vnode<N>(D, m, pt)], vg);
    }
    qn[f] = vq;
    gn[f] = vg;
  }
}

// chunk_trace2 for even N by partner-lane pairs (as chunk_trace_x2 in
// stage_nb.h): lanes 2k and 2k + 1 hold x-adjacent points whose line nodes
// form a 16-byte pair at every m; each lane loads the Q and gR pairs at
// m = 2j + (pt & 1) and takes the other m from its partner by DPP.  Same
// FMA chains as chunk_trace2.  Both lanes of a pair must be active.
template <int N, int D>
__device__ __forceinline__ void chunk_trace2_x2(const double* __restrict__ Q, const double* __restrict__ G,
                                                int64_t EN3, int64_t cofs, int pt, const double* cq,
                                                const double* cg, double* qn, double* gn) {
  static_assert(N % 2 == 0, "pairs of x-adjacent points need an even N");
  const int s = pt & 1;
  const int pe = pt - s;
  double2 wq[5][N / 2], wg[5][N / 2];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
#pragma unroll
    for (int j = 0; j < N / 2; ++j) {
      const int64_t o = f * EN3 + cofs + (s ? vnode<N>(D, 2 * j + 1, pe) : vnode<N>(D, 2 * j, pe));
      __builtin_memcpy(&wq[f][j], Q + o, 16);
      __builtin_memcpy(&wg[f][j], G + o, 16);
    }
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    double vq = 0.0, vg = 0.0;
#pragma unroll
    for (int j = 0; j < N / 2; ++j) {
      const double pqx = dgdev::swap_adjacent(wq[f][j].x), pqy = dgdev::swap_adjacent(wq[f][j].y);
      const double pgx = dgdev::swap_adjacent(wg[f][j].x), pgy = dgdev::swap_adjacent(wg[f][j].y);
      vq = fma(cq[2 * j], s ? pqy : wq[f][j].x, vq);
      vg = fma(cg[2 * j], s ? pgy : wg[f][j].x, vg);
      vq = fma(cq[2 * j + 1], s ? wq[f][j].y : pqx, vq);
      vg = fma(cg[2 * j + 1], s ? wg[f][j].y : pgx, vg);
    }
    qn[f] = vq;
    gn[f] = vg;
  }
}

// Adjoint of this element's side of face (D, SIDE) at point pt: own traces
// from LDS (sQ, sG slot `so`), the neighbour's from LDS (slot `sn`, x-faces)
// or from registers.
template <int N, int D, int SIDE, bool LDSNB>
__device__ __forceinline__ void face_vjp(const double* sQ, const double* sG, int so, int sn, const double* qnr,
                                         const double* gnr, int NH, int pt, const double* sLm, const double* sLp,
                                         const double* sLiftm, const double* sLiftp, double sc, double gamma,
                                         double gm1, double* gq) {
  constexpr int N3 = N * N * N;
  double qo[5], go[5], qn[5], gn[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    qo[f] = line_sum<N>(sQ + f * NH + so * N3, SIDE ? sLp : sLm, D, pt);
    go[f] = line_sum<N>(sG + f * NH + so * N3, SIDE ? sLiftp : sLiftm, D, pt);
    qn[f] = LDSNB ? line_sum<N>(sQ + f * NH + sn * N3, SIDE ? sLm : sLp, D, pt) : qnr[f];
    gn[f] = LDSNB ? line_sum<N>(sG + f * NH + sn * N3, SIDE ? sLiftm : sLiftp, D, pt) : gnr[f];
  }
  double gf[5], qm[5], qp[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    gf[f] = SIDE ? sc * (gn[f] - go[f]) : sc * (go[f] - gn[f]);
    qm[f] = SIDE ? qo[f] : qn[f];
    qp[f] = SIDE ? qn[f] : qo[f];
  }
  lf_vjp_d<D>(qm, qp, gamma, gm1, gf, SIDE != 0, gq);
}

template <int N>
__global__ void __launch_bounds__(VCfg<N>::NT)
k_vjp_nb(DGTables tb, const double* __restrict__ Q, const double* __restrict__ gR, double* __restrict__ gQ,
         DGOrder ord) {
  constexpr int EPB = VCfg<N>::EPB, NT = VCfg<N>::NT;
  constexpr int N2 = N * N, N3 = N2 * N, NODES = EPB * N3, FP = EPB * N2, NH = (EPB + 2) * N3;
  constexpr int NW = NT / 64;
  using S = dgdev::FaceSlots<N, EPB>;
  constexpr int RND = (S::NS + NW - 1) / NW;
  constexpr int RNDG = (S::NYZ + NW - 1) / NW;
  constexpr int HPT = (2 * N3 + NT - 1) / NT;
  static_assert(NODES <= NT, "one thread per node");
  __shared__ double smem[VjpSmem<N, EPB>::size];
  double* sQ = smem;            // [5][NH] slot 0 left neighbour, 1..ne own, ne+1 right neighbour
  double* sG = sQ + 5 * NH;     // [5][NH]
  double* sH = sG + 5 * NH;     // [6][5][FP] face adjoints gq
  double* sDh = sH + 30 * FP;
  double* sLm = sDh + N * N;
  double* sLp = sLm + N;
  double* sLiftm = sLp + N;
  double* sLiftp = sLiftm + N;

  const int tid = threadIdx.x;
  int e0, ne;
  dgdev::block_elements<EPB>(tb, ord, blockIdx.x, gridDim.x, e0, ne);
  const int nx = tb.nx, ny = tb.ny, nz = tb.nz;
  const int64_t EN3 = (int64_t)tb.E * N3;
  const int row = e0 / nx;
  const int x0 = e0 - row * nx;
  const int ey = row % ny, ez = row / ny;
  const int plane = nx * ny;
  const int eym = ey == 0 ? e0 + (ny - 1) * nx : e0 - nx;
  const int eyp = ey == ny - 1 ? e0 - (ny - 1) * nx : e0 + nx;
  const int ezm = ez == 0 ? e0 + (nz - 1) * plane : e0 - plane;
  const int ezp = ez == nz - 1 ? e0 - (nz - 1) * plane : e0 + plane;
  const int exl = x0 == 0 ? e0 + nx - 1 : e0 - 1;
  const int exr = x0 + ne == nx ? e0 - x0 : e0 + ne;
  double lmr[N], lpr[N], lfm[N], lfp[N];
#pragma unroll
  for (int m = 0; m < N; ++m) {
    lmr[m] = tb.lm[m];
    lpr[m] = tb.lp[m];
    lfm[m] = tb.liftm[m];
    lfp[m] = tb.liftp[m];
  }

  // ---- A: all loads before the first wait (unconditional; absent points
  //         read the block's first node)
  const bool nthr = tid < NODES;
  const int el = tid / N3;
  const int t = tid - el * N3;
  const int ni = t % N, nj = (t / N) % N, nk = t / N2;
  const bool act = nthr && el < ne;
  const int64_t gofs = (int64_t)e0 * N3 + tid;
  const int64_t lofs = act ? gofs : (int64_t)e0 * N3;
  double q[5], g[5], hq[HPT][5], hg[HPT][5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    q[f] = Q[f * EN3 + lofs];
    g[f] = gR[f * EN3 + lofs];
  }
#pragma unroll
  for (int h = 0; h < HPT; ++h) {
    const int xh = tid + h * NT;
    const int x = xh < 2 * N3 ? xh : 0;
    const int right = x >= N3;
    const int64_t hofs = (int64_t)(right ? exr : exl) * N3 + (x - right * N3);
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      hq[h][f] = Q[f * EN3 + hofs];
      hg[h][f] = gR[f * EN3 + hofs];
    }
  }
  const int wave = tid >> 6, lane = tid & 63;
  double qnb[RNDG][5], gnb[RNDG][5];
#pragma unroll
  for (int u = 0; u < RNDG; ++u) {
    const int s = wave + u * NW;
    const int i = (s < S::NYZ ? S::chunk(s) : 0) * 64 + lane;
    const int fel = i / N2, pt = i - fel * N2;
    if (s < S::NYZ && i < FP && fel < ne) {
      if constexpr (N == 4) {
        // partner-lane pairs (lanes of a pair share fel, FP is even)
        switch (S::face(s)) {   // uniform over the wave; neighbour's face on the other side
          case 2: chunk_trace2_x2<N, 1>(Q, gR, EN3, (int64_t)(eym + fel) * N3, pt, lpr, lfp, qnb[u], gnb[u]); break;
          case 3: chunk_trace2_x2<N, 1>(Q, gR, EN3, (int64_t)(eyp + fel) * N3, pt, lmr, lfm, qnb[u], gnb[u]); break;
          case 4: chunk_trace2_x2<N, 2>(Q, gR, EN3, (int64_t)(ezm + fel) * N3, pt, lpr, lfp, qnb[u], gnb[u]); break;
          default: chunk_trace2_x2<N, 2>(Q, gR, EN3, (int64_t)(ezp + fel) * N3, pt, lmr, lfm, qnb[u], gnb[u]); break;
        }
      } else {
        switch (S::face(s)) {   // uniform over the wave; neighbour's face on the other side
          case 2: chunk_trace2<N, 1>(Q, gR, EN3, (int64_t)(eym + fel) * N3, pt, lpr, lfp, qnb[u], gnb[u]); break;
          case 3: chunk_trace2<N, 1>(Q, gR, EN3, (int64_t)(eyp + fel) * N3, pt, lmr, lfm, qnb[u], gnb[u]); break;
          case 4: chunk_trace2<N, 2>(Q, gR, EN3, (int64_t)(ezm + fel) * N3, pt, lpr, lfp, qnb[u], gnb[u]); break;
          default: chunk_trace2<N, 2>(Q, gR, EN3, (int64_t)(ezp + fel) * N3, pt, lmr, lfm, qnb[u], gnb[u]); break;
        }
      }
    } else {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        qnb[u][f] = f == 0 ? 1.0 : (f == 4 ? 2.5 : 0.0);
        gnb[u][f] = 0.0;
      }
    }
  }
  // tables from uniform (scalar) kernarg reads
  if (tid < N * N) {
    double v = 0.0;
#pragma unroll
    for (int x = 0; x < N * N; ++x) v = tid == x ? tb.Dh[x] : v;
    sDh[tid] = v;
  }
  if (tid < N) {
    double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      a = tid == m ? tb.lm[m] : a;
      b = tid == m ? tb.lp[m] : b;
      c = tid == m ? tb.liftm[m] : c;
      d = tid == m ? tb.liftp[m] : d;
    }
    sLm[tid] = a;
    sLp[tid] = b;
    sLiftm[tid] = c;
    sLiftp[tid] = d;
  }
  if (act) {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      sQ[f * NH + N3 + tid] = q[f];
      sG[f * NH + N3 + tid] = g[f];
    }
  }
#pragma unroll
  for (int h = 0; h < HPT; ++h) {
    const int x = tid + h * NT;
    if (x < 2 * N3) {
      const int right = x >= N3;
      const int o = (right ? ne + 1 : 0) * N3 + (x - right * N3);
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        sQ[f * NH + o] = hq[h][f];
        sG[f * NH + o] = hg[h][f];
      }
    }
  }
  __syncthreads();

  // ---- B: adjoint of this element's side of every face
#pragma unroll
  for (int u = 0; u < RND; ++u) {
    const int s = wave + u * NW;
    const int i = (s < S::NS ? S::chunk(s) : 0) * 64 + lane;
    if (s < S::NS && i < FP) {
      const int face = S::face(s);
      const int fel = i / N2, pt = i - fel * N2;
      const int so = fel + 1;
      const double* qv = qnb[u < RNDG ? u : 0];
      const double* gv = gnb[u < RNDG ? u : 0];
      const double ga = tb.gamma, g1 = tb.gm1;
      double gq[5];
      switch (face) {   // uniform over the wave
        case 0:
          face_vjp<N, 0, 0, true>(sQ, sG, so, so - 1, qv, gv, NH, pt, sLm, sLp, sLiftm, sLiftp, tb.sc[0], ga, g1, gq);
          break;
        case 1:
          face_vjp<N, 0, 1, true>(sQ, sG, so, so + 1, qv, gv, NH, pt, sLm, sLp, sLiftm, sLiftp, tb.sc[0], ga, g1, gq);
          break;
        case 2:
          face_vjp<N, 1, 0, false>(sQ, sG, so, so, qv, gv, NH, pt, sLm, sLp, sLiftm, sLiftp, tb.sc[1], ga, g1, gq);
          break;
        case 3:
          face_vjp<N, 1, 1, false>(sQ, sG, so, so, qv, gv, NH, pt, sLm, sLp, sLiftm, sLiftp, tb.sc[1], ga, g1, gq);
          break;
        case 4:
          face_vjp<N, 2, 0, false>(sQ, sG, so, so, qv, gv, NH, pt, sLm, sLp, sLiftm, sLiftp, tb.sc[2], ga, g1, gq);
          break;
        default:
          face_vjp<N, 2, 1, false>(sQ, sG, so, so, qv, gv, NH, pt, sLm, sLp, sLiftm, sLiftp, tb.sc[2], ga, g1, gq);
          break;
      }
#pragma unroll
      for (int f = 0; f < 5; ++f) sH[(face * 5 + f) * FP + i] = gq[f];
    }
  }
  __syncthreads();

  // ---- C: volume (transposed contraction, flux Jacobian transpose) and the
  //         face adjoints lifted back onto the lines
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int m = d == 0 ? ni : (d == 1 ? nj : nk);
    const int pt = d == 0 ? nj + N * nk : (d == 1 ? ni + N * nk : ni + N * nj);
    const double sc = tb.sc[d];
    const double* gline = sG + (el + 1) * N3;
    double gF[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      double sacc = 0.0;
#pragma unroll
      for (int i2 = 0; i2 < N; ++i2) sacc = fma(sDh[i2 * N + m], gline[f * NH + vnode<N>(d, i2, pt)], sacc);
      gF[f] = sc * sacc;
    }
    if (d == 0) flux_vjp<0>(q, gF, tb.gm1, acc);
    else if (d == 1) flux_vjp<1>(q, gF, tb.gm1, acc);
    else flux_vjp<2>(q, gF, tb.gm1, acc);
#pragma unroll
    for (int f = 0; f < 5; ++f)
      acc[f] += sLp[m] * sH[((2 * d + 1) * 5 + f) * FP + el * N2 + pt] + sLm[m] * sH[((2 * d) * 5 + f) * FP + el * N2 + pt];
  }
  if (act) {
#pragma unroll
    for (int f = 0; f < 5; ++f) gQ[f * EN3 + gofs] = acc[f];
  }
}

// gtot = gres + b * gQ (state-sized axpy for the reverse RK stage).
__global__ void __launch_bounds__(256)
k_axpy(int64_t n, const double* __restrict__ x, double b, const double* __restrict__ y, double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = fma(b, y[i], x[i]);
}

// gQ += dt * v ; gres = a * gtot
__global__ void __launch_bounds__(256)
k_rk_reverse(int64_t n, const double* __restrict__ v, double dt, double a, const double* __restrict__ gtot,
             double* __restrict__ gQ, double* __restrict__ gres) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    gQ[i] = fma(dt, v[i], gQ[i]);
    gres[i] = a * gtot[i];
  }
}

// Gradient of the kinetic-energy integral sum_e J sum_q w_q |m_q|^2 / (2 rho_q)
// (the nodal Gauss-Legendre rule of the domain integrals) with respect to
// every nodal value: d/d rho = -|u|^2/2 Jw, d/d m_d = u_d Jw, d/d (rho E) = 0,
// with u = m / rho and Jw = J w_i w_j w_k of the node.
template <int N>
__global__ void __launch_bounds__(256)
k_ke_grad(DGTables tb, const double* __restrict__ Q, double* __restrict__ G) {
  constexpr int N3 = N * N * N;
  const int64_t total = (int64_t)tb.E * N3;
  for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < total; g += (int64_t)gridDim.x * 256) {
    const int t = (int)(g % N3);
    const int i = t % N, j = (t / N) % N, k = t / (N * N);
    const double jw = tb.J * tb.w[i] * tb.w[j] * tb.w[k];
    const double rinv = 1.0 / Q[g];
    const double u = Q[total + g] * rinv, v = Q[2 * total + g] * rinv, w = Q[3 * total + g] * rinv;
    G[g] = -0.5 * (u * u + v * v + w * w) * jw;
    G[total + g] = u * jw;
    G[2 * total + g] = v * jw;
    G[3 * total + g] = w * jw;
    G[4 * total + g] = 0.0;
  }
}

template <int N>
int launch_ke_grad_n(const dg_ctx* c, const double* Q, double* G) {
  const int64_t blocks64 = (c->E * N * N * N + 255) / 256;
  const unsigned grid = (unsigned)(blocks64 < 65536 ? (blocks64 > 0 ? blocks64 : 1) : 65536);
  hipLaunchKernelGGL(k_ke_grad<N>, dim3(grid), dim3(256), 0, c->stream, c->tab, Q, G);
  return (int)hipGetLastError();
}

template <int N>
int launch_vjp_n(const dg_ctx* c, const double* Q, const double* gR, double* gQ, double* TQ, double* TG) {
  constexpr int EPB = VCfg<N>::EPB;
  const unsigned grid = (unsigned)((c->E + EPB - 1) / EPB);
  const dim3 blk(VCfg<N>::NT);
  hipLaunchKernelGGL((k_vtrace<N, false>), dim3(grid), blk, 0, c->stream, c->tab, Q, TQ);
  hipLaunchKernelGGL((k_vtrace<N, true>), dim3(grid), blk, 0, c->stream, c->tab, gR, TG);
  hipLaunchKernelGGL(k_vjp<N>, dim3(grid), blk, 0, c->stream, c->tab, Q, gR, TQ, TG, gQ);
  return (int)hipGetLastError();
}

template <int N>
int launch_vjp_nb_n(const dg_ctx* c, const double* Q, const double* gR, double* gQ) {
  unsigned grid;
  const DGOrder ord = dg_order(c, VCfg<N>::EPB, &grid);
  hipLaunchKernelGGL(k_vjp_nb<N>, dim3(grid), dim3(VCfg<N>::NT), 0, c->stream, c->tab, Q, gR, gQ, ord);
  return (int)hipGetLastError();
}

}  // namespace

int dg_launch_vjp(const dg_ctx* c, const double* Q, const double* gR, double* gQ, char* ws) {
  if (c->exchange == DG_EXCHANGE_NEIGHBOUR) {
    switch (c->N) {
      case 1: return launch_vjp_nb_n<1>(c, Q, gR, gQ);
      case 2: return launch_vjp_nb_n<2>(c, Q, gR, gQ);
      case 3: return launch_vjp_nb_n<3>(c, Q, gR, gQ);
      case 4: return launch_vjp_nb_n<4>(c, Q, gR, gQ);
      case 5: return launch_vjp_nb_n<5>(c, Q, gR, gQ);
      case 6: return launch_vjp_nb_n<6>(c, Q, gR, gQ);
      case 7: return launch_vjp_nb_n<7>(c, Q, gR, gQ);
      case 8: return launch_vjp_nb_n<8>(c, Q, gR, gQ);
      default: return (int)hipErrorInvalidValue;
    }
  }
  const DGWorkspace L = dg_workspace_layout(c);
  double* TQ = (double*)(ws + L.off_trace0);
  double* TG = (double*)(ws + L.off_trace1);
  switch (c->N) {
    case 1: return launch_vjp_n<1>(c, Q, gR, gQ, TQ, TG);
    case 2: return launch_vjp_n<2>(c, Q, gR, gQ, TQ, TG);
    case 3: return launch_vjp_n<3>(c, Q, gR, gQ, TQ, TG);
    case 4: return launch_vjp_n<4>(c, Q, gR, gQ, TQ, TG);
    case 5: return launch_vjp_n<5>(c, Q, gR, gQ, TQ, TG);
    case 6: return launch_vjp_n<6>(c, Q, gR, gQ, TQ, TG);
    case 7: return launch_vjp_n<7>(c, Q, gR, gQ, TQ, TG);
    case 8: return launch_vjp_n<8>(c, Q, gR, gQ, TQ, TG);
    default: return (int)hipErrorInvalidValue;
  }
}

int dg_launch_axpy(const dg_ctx* c, int64_t n, const double* x, double b, const double* y, double* out) {
  const int64_t blocks64 = (n + 255) / 256;
  const unsigned grid = (unsigned)(blocks64 < 65536 ? (blocks64 > 0 ? blocks64 : 1) : 65536);
  hipLaunchKernelGGL(k_axpy, dim3(grid), dim3(256), 0, c->stream, n, x, b, y, out);
  return (int)hipGetLastError();
}

int dg_launch_rk_reverse(const dg_ctx* c, int64_t n, const double* v, double dt, double a, const double* gtot,
                         double* gQ, double* gres) {
  const int64_t blocks64 = (n + 255) / 256;
  const unsigned grid = (unsigned)(blocks64 < 65536 ? (blocks64 > 0 ? blocks64 : 1) : 65536);
  hipLaunchKernelGGL(k_rk_reverse, dim3(grid), dim3(256), 0, c->stream, n, v, dt, a, gtot, gQ, gres);
  return (int)hipGetLastError();
}

int dg_launch_ke_grad(const dg_ctx* c, const double* Q, double* G) {
  switch (c->N) {
    case 1: return launch_ke_grad_n<1>(c, Q, G);
    case 2: return launch_ke_grad_n<2>(c, Q, G);
    case 3: return launch_ke_grad_n<3>(c, Q, G);
    case 4: return launch_ke_grad_n<4>(c, Q, G);
    case 5: return launch_ke_grad_n<5>(c, Q, G);
    case 6: return launch_ke_grad_n<6>(c, Q, G);
    case 7: return launch_ke_grad_n<7>(c, Q, G);
    case 8: return launch_ke_grad_n<8>(c, Q, G);
    default: return (int)hipErrorInvalidValue;
  }
}
