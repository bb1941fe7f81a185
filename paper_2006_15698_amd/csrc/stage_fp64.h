// Device code of the fused FP64 DG Euler stage, shared by the single-mesh
// kernels (kern_fp64.hip) and the batched persistent kernel (kern_batch.hip).
//
// One workgroup of NT threads owns EPB consecutive elements of one mesh, one
// thread per node (Section IV: fine-grain parallelism inside an element).
//   A. load Q (and res) once, coalesced along the SoA layout; stage Q in LDS;
//      prefetch the neighbours' face traces written by the previous launch
//   B. local Lax-Friedrichs flux at every face point of the six faces of
//      every element (own trace interpolated from LDS, Section II-B)
//   C. per direction: pointwise Euler flux F^d (Eq. (2)) into LDS, 1-D
//      sum-factorised volume contraction along the line of the node plus
//      the lift of the two face fluxes on that line (Eq. (5) with the
//      diagonal collocated mass matrix divided out)
//   D. RK axpy in registers (Sections IV-V), store Q and res, then
//      interpolate the updated Q to the six faces and store those traces for
//      the next stage's neighbours.
#pragma once

#include "dg_internal.h"

namespace dgdev {

// Node index inside an element of the point with index m along direction d
// and tangential index pt = a + N b (lower tangential axis fastest).
template <int N>
__host__ __device__ __forceinline__ int tnode(int d, int m, int pt) {
  if (d == 0) return pt * N + m;                          // i = m, j = a, k = b
  if (d == 1) return (pt / N) * N * N + m * N + (pt % N); // j = m, i = a, k = b
  return m * N * N + pt;                                   // k = m, i = a, j = b
}

// Periodic neighbour of element e one step along direction d (dir = +-1).
__device__ __forceinline__ int neighbour(int nx, int ny, int nz, int e, int d, int dir) {
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

// Local Lax-Friedrichs flux across a face with normal +e_D (Section II-B):
// F* = (F^D(qm) + F^D(qp))/2 - lambda/2 (qp - qm),
// lambda = max(|u_D-| + c-, |u_D+| + c+).  Ties pick the - side.  The
// direction is a template parameter so that every array index is static
// (a runtime index would force qm/qp into scratch memory).
// 1/a: the hardware reciprocal estimate refined by two Newton-Raphson steps
// r <- r + r (1 - a r) in FMA form, about half the instructions of a division.  On the 2^22 seeded
// inputs of the library's accuracy check (dg_recip_sqrt: log-uniform in
// [2^-12, 2^12], near 1, powers of two, 60..120) it equals the correctly
// rounded quotient bit for bit.  A zero or non-finite input gives NaN or
// infinity, as the state is then non-physical anyway.
__device__ __forceinline__ double recip(double a) {
  double r = __builtin_amdgcn_rcp(a);
  double e = fma(-a, r, 1.0);
  r = fma(r, e, r);
  e = fma(-a, r, 1.0);
  return fma(r, e, r);
}

// sqrt(x) for x >= 0: from the reciprocal-square-root estimate y, one
// coupled Newton step on g = x y ~ sqrt(x) and h = y/2 ~ 1/(2 sqrt(x)) (the
// FMA square-root iteration described by Markstein for IA-64), then a final
// correction of g with the residual x - g^2 (0 for x = 0).  Equal to
// the correctly rounded square root bit for bit on the same checked inputs.
__device__ __forceinline__ double root(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double t = fma(-g, h, 0.5);
  g = fma(g, t, g);
  h = fma(h, t, h);
  const double d = fma(-g, g, x);
  const double r = fma(d, h, g);
  return x == 0.0 ? 0.0 : r;
}

template <int D>
__device__ __forceinline__ void lf_flux_d(const double* qm, const double* qp, double gamma, double gm1,
                                          double* out) {
  const double rm = recip(qm[0]);
  const double rp = recip(qp[0]);
  const double unm = qm[1 + D] * rm;
  const double unp = qp[1 + D] * rp;
  const double pm = gm1 * (qm[4] - 0.5 * (qm[1] * qm[1] + qm[2] * qm[2] + qm[3] * qm[3]) * rm);
  const double pp = gm1 * (qp[4] - 0.5 * (qp[1] * qp[1] + qp[2] * qp[2] + qp[3] * qp[3]) * rp);
  const double lm = fabs(unm) + root(gamma * pm * rm);
  const double lp = fabs(unp) + root(gamma * pp * rp);
  const double lam = lm >= lp ? lm : lp;
  double fm[5], fp[5];
  fm[0] = qm[1 + D];
  fp[0] = qp[1 + D];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    fm[1 + k] = qm[1 + k] * unm + (k == D ? pm : 0.0);
    fp[1 + k] = qp[1 + k] * unp + (k == D ? pp : 0.0);
  }
  fm[4] = (qm[4] + pm) * unm;
  fp[4] = (qp[4] + pp) * unp;
#pragma unroll
  for (int f = 0; f < 5; ++f) out[f] = 0.5 * (fm[f] + fp[f]) - 0.5 * lam * (qp[f] - qm[f]);
}

__device__ __forceinline__ void lf_flux(const double* qm, const double* qp, int d, double gamma, double gm1,
                                        double* out) {
  if (d == 0) lf_flux_d<0>(qm, qp, gamma, gm1, out);
  else if (d == 1) lf_flux_d<1>(qm, qp, gamma, gm1, out);
  else lf_flux_d<2>(qm, qp, gamma, gm1, out);
}

// Trace of one field on face (d, side) at tangential point pt: sum over the
// normal line of l_m(+-1) Q_m, as an explicit FMA chain so that every kernel
// that produces traces rounds identically.
template <int N>
__device__ __forceinline__ double line_trace(const double* sq, const double* coef, int d, int pt) {
  double v = 0.0;
#pragma unroll
  for (int m = 0; m < N; ++m) v = fma(coef[m], sq[tnode<N>(d, m, pt)], v);
  return v;
}

// Shared-memory footprint (doubles) of the FP64 stage body.
template <int N, int EPB>
struct Fp64Smem {
  static constexpr int NODES = EPB * N * N * N;
  static constexpr int FP = EPB * N * N;
  static constexpr int size = 10 * NODES + 30 * FP + N * N + 4 * N;
};

// Traces of the element states in sQ ([5][NODES]) for elements e0.. of a
// mesh with E elements, written to T[(face*5+f)][E][N^2].
template <int N, int EPB, int NT>
__device__ __forceinline__ void write_traces(const double* sQ, const double* sLm, const double* sLp, int e0,
                                             int E, double* __restrict__ T, int tid) {
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr int NODES = EPB * N3, FP = EPB * N2;
  const int64_t EN2 = (int64_t)E * N2;
  for (int it = tid; it < 30 * FP; it += NT) {
    const int pt = it % N2;
    const int r1 = it / N2;
    const int fel = r1 % EPB;
    const int r2 = r1 / EPB;
    const int f = r2 % 5;
    const int face = r2 / 5;
    const int ee = e0 + fel;
    if (ee >= E) continue;
    const double* coef = (face & 1) ? sLp : sLm;
    T[(int64_t)(face * 5 + f) * EN2 + (int64_t)ee * N2 + pt] =
        line_trace<N>(sQ + f * NODES + fel * N3, coef, face >> 1, pt);
  }
}

// Shared-memory footprint (doubles) of the trace body.
template <int N, int EPB>
struct TraceSmem {
  static constexpr int size = 5 * EPB * N * N * N + 2 * N;
};

// Face traces of elements e0..e0+EPB-1 of Q.  smem: TraceSmem<N,EPB>::size.
template <int N, int EPB, int NT>
__device__ __forceinline__ void trace_body(const DGTables& tb, const double* __restrict__ Q, double* __restrict__ T,
                                           int e0, double* smem, int tid) {
  constexpr int N3 = N * N * N, NODES = EPB * N3;
  double* sQ = smem;
  double* sLm = smem + 5 * NODES;
  double* sLp = sLm + N;
  const int E = tb.E;
  const int64_t EN3 = (int64_t)E * N3;
  if (tid < N) {
    sLm[tid] = tb.lm[tid];
    sLp[tid] = tb.lp[tid];
  }
  for (int x = tid; x < NODES; x += NT) {
    if (e0 + x / N3 < E) {
#pragma unroll
      for (int f = 0; f < 5; ++f) sQ[f * NODES + x] = Q[f * EN3 + (int64_t)e0 * N3 + x];
    }
  }
  __syncthreads();
  write_traces<N, EPB, NT>(sQ, sLm, sLp, e0, E, T, tid);
}

// One fused stage for elements e0..e0+EPB-1.  MODE 0: RR = dQ/dt.  MODE 1:
// RK stage in place (RR = res).  MODE 2: RK stage plus the traces of the
// updated Q into Tout.  smem: Fp64Smem<N,EPB>::size doubles.
template <int N, int MODE, int EPB, int NT>
__device__ __forceinline__ void stage_body(const DGTables& tb, double* __restrict__ Q, double* __restrict__ RR,
                                           const double* __restrict__ Tin, double* __restrict__ Tout, double rka,
                                           double rkb, double dt, int first, int e0, double* smem, int tid) {
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr int NODES = EPB * N3, FP = EPB * N2;
  constexpr int NITEM = 6 * FP;
  constexpr int IPT = (NITEM + NT - 1) / NT;
  static_assert(NODES <= NT, "one thread per node");

  double* sQ = smem;                 // [5][NODES]
  double* sF = sQ + 5 * NODES;       // [5][NODES]
  double* sH = sF + 5 * NODES;       // [6][5][FP]
  double* sDh = sH + 30 * FP;        // [N][N]
  double* sLm = sDh + N * N;
  double* sLp = sLm + N;
  double* sLiftm = sLp + N;
  double* sLiftp = sLiftm + N;

  const int E = tb.E;
  const int64_t EN3 = (int64_t)E * N3;
  const int64_t EN2 = (int64_t)E * N2;

  for (int x = tid; x < N * N; x += NT) sDh[x] = tb.Dh[x];
  if (tid < N) {
    sLm[tid] = tb.lm[tid];
    sLp[tid] = tb.lp[tid];
    sLiftm[tid] = tb.liftm[tid];
    sLiftp[tid] = tb.liftp[tid];
  }

  // ---- A: this thread's node
  const bool nthr = tid < NODES;
  const int el = tid / N3;
  const int t = tid - el * N3;
  const int ni = t % N, nj = (t / N) % N, nk = t / N2;
  const int e = e0 + el;
  const bool act = nthr && e < E;
  const int64_t gofs = (int64_t)e * N3 + t;
  double q[5], r[5];
  if (act) {
#pragma unroll
    for (int f = 0; f < 5; ++f) q[f] = Q[f * EN3 + gofs];
  } else {
    q[0] = 1.0; q[1] = 0.0; q[2] = 0.0; q[3] = 0.0; q[4] = 2.5;
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) r[f] = 0.0;
  if (MODE != 0 && act && !first) {
#pragma unroll
    for (int f = 0; f < 5; ++f) r[f] = RR[f * EN3 + gofs];
  }
  if (nthr) {
#pragma unroll
    for (int f = 0; f < 5; ++f) sQ[f * NODES + tid] = q[f];
  }
  // neighbours' traces for this thread's face items
  double nb[IPT][5];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int it = tid + u * NT;
    const int face = it / FP;
    const int rem = it - face * FP;
    const int fel = rem / N2;
    const int pt = rem - fel * N2;
    const int ee = e0 + fel;
    if (it < NITEM && ee < E) {
      const int d = face >> 1, side = face & 1;
      const int nbe = neighbour(tb.nx, tb.ny, tb.nz, ee, d, side ? 1 : -1);
      const int oface = 2 * d + (1 - side);
#pragma unroll
      for (int f = 0; f < 5; ++f) nb[u][f] = Tin[(int64_t)(oface * 5 + f) * EN2 + (int64_t)nbe * N2 + pt];
    } else {
      nb[u][0] = 1.0; nb[u][1] = 0.0; nb[u][2] = 0.0; nb[u][3] = 0.0; nb[u][4] = 2.5;
    }
  }
  __syncthreads();

  // ---- B: Lax-Friedrichs flux at every face point
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int it = tid + u * NT;
    if (it < NITEM) {
      const int face = it / FP;
      const int rem = it - face * FP;
      const int fel = rem / N2;
      const int pt = rem - fel * N2;
      const int d = face >> 1, side = face & 1;
      double own[5], fs[5];
      const double* coef = side ? sLp : sLm;
#pragma unroll
      for (int f = 0; f < 5; ++f) own[f] = line_trace<N>(sQ + f * NODES + fel * N3, coef, d, pt);
      // select values (not pointers) so that nb and own stay in registers
      double qm[5], qp[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        qm[f] = side ? own[f] : nb[u][f];
        qp[f] = side ? nb[u][f] : own[f];
      }
      lf_flux(qm, qp, d, tb.gamma, tb.gm1, fs);
#pragma unroll
      for (int f = 0; f < 5; ++f) sH[(face * 5 + f) * FP + fel * N2 + pt] = fs[f];
    }
  }

  // ---- C: volume contraction + lift, one direction at a time
  const double rinv = recip(q[0]);
  const double pr = tb.gm1 * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) * rinv);
  double acc[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) acc[f] = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double ud = q[1 + d] * rinv;
    if (nthr) {
      sF[0 * NODES + tid] = q[1 + d];
      sF[1 * NODES + tid] = q[1] * ud + (d == 0 ? pr : 0.0);
      sF[2 * NODES + tid] = q[2] * ud + (d == 1 ? pr : 0.0);
      sF[3 * NODES + tid] = q[3] * ud + (d == 2 ? pr : 0.0);
      sF[4 * NODES + tid] = (q[4] + pr) * ud;
    }
    __syncthreads();
    if (nthr) {
      const int m = d == 0 ? ni : (d == 1 ? nj : nk);
      const int pt = d == 0 ? nj + N * nk : (d == 1 ? ni + N * nk : ni + N * nj);
      const double sc = tb.sc[d];
      const double lfm = sLiftm[m], lfp = sLiftp[m];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) s = fma(sDh[m * N + a], sF[f * NODES + el * N3 + tnode<N>(d, a, pt)], s);
        s = fma(lfm, sH[((2 * d) * 5 + f) * FP + el * N2 + pt], s);
        s = fma(-lfp, sH[((2 * d + 1) * 5 + f) * FP + el * N2 + pt], s);
        acc[f] = fma(sc, s, acc[f]);
      }
    }
    if (d < 2) __syncthreads();
  }

  // ---- D: output
  if (MODE == 0) {
    if (act) {
#pragma unroll
      for (int f = 0; f < 5; ++f) RR[f * EN3 + gofs] = acc[f];
    }
  } else {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      r[f] = first ? dt * acc[f] : fma(rka, r[f], dt * acc[f]);
      q[f] = fma(rkb, r[f], q[f]);
    }
    if (act) {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        Q[f * EN3 + gofs] = q[f];
        RR[f * EN3 + gofs] = r[f];
      }
    }
    if (MODE == 2) {
      // sQ was last read in phase B, which every thread finished before the
      // first barrier of phase C.
      if (nthr) {
#pragma unroll
        for (int f = 0; f < 5; ++f) sQ[f * NODES + tid] = q[f];
      }
      __syncthreads();
      write_traces<N, EPB, NT>(sQ, sLm, sLp, e0, E, Tout, tid);
    }
  }
}

}  // namespace dgdev
