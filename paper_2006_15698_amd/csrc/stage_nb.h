// Device code of the FP64 DG Euler stage with neighbour reads.
//
// Same arithmetic as stage_body (stage_fp64.h), but the trace of a
// neighbour on the shared face is interpolated directly from the
// neighbour's state (sum over its normal line of l_m(-+1) Q_m, the same
// FMA chain as line_trace) instead of being read from a trace buffer that
// the previous launch wrote.  The state is read from Qin and the updated
// state written to Qout (a different buffer), so no launch reads what it
// writes.  Per node and stage HBM traffic is Q in, res in, Q out, res out
// (160 B) plus whatever neighbour reads miss the caches; there are no trace
// buffers.  Results are bitwise those of stage_body.
#pragma once

#include "stage_fp64.h"

namespace dgdev {

// Workgroup -> element block mapping that gives each XCD a contiguous range
// of blocks: workgroups are dispatched round robin over the 8 XCDs, so
// workgroup w runs on XCD w % 8; its block is the (w / 8)-th of that XCD's
// slab.  A bijection on [0, nblk) for any nblk.
__host__ __device__ __forceinline__ int xcd_block(int w, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = w & 7, i = w >> 3;
  return x * q + (x < r ? x : r) + i;
}

__host__ __device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

// Elements [e0, e0 + ne) of workgroup w of nblk under the visiting order o
// (see DGOrder).  Every value is uniform over the workgroup.

template <int EPB>
__host__ __device__ __forceinline__ void block_elements(const DGTables& tb, const DGOrder& o, int w, int nblk,
                                                        int& e0, int& ne) {
  const int s = o.xcd ? xcd_block(w, nblk) : w;
  if (!o.pencil) {
    e0 = s * EPB;
    ne = imin(EPB, tb.E - e0);
    return;
  }
  const int slab = o.nxb * tb.ny * o.tz;     // blocks of a full z-slab
  const int pz = s / slab;
  int r = s - pz * slab;
  const int tz = imin(o.tz, tb.nz - pz * o.tz);
  const int pen = tb.ny * tz * o.tx;         // blocks of a full pencil of this slab
  const int px = r / pen;
  r -= px * pen;
  const int tx = imin(o.tx, o.nxb - px * o.tx);
  const int y = r / (tz * tx);
  r -= y * (tz * tx);
  const int zz = r / tx;
  const int x0 = (px * o.tx + r - zz * tx) * EPB;
  e0 = ((pz * o.tz + zz) * tb.ny + y) * tb.nx + x0;
  ne = imin(EPB, tb.nx - x0);
}

// Streamed loads and stores; non-temporal when `nt` (uniform).
__device__ __forceinline__ double ld_stream(const double* p, bool nt) {
  return nt ? __builtin_nontemporal_load(p) : *p;
}
__device__ __forceinline__ void st_stream(double* p, double v, bool nt) {
  if (nt)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Elements [e0, e0 + ne) with ne <= EPB.  MODE 0: RR = dQ/dt (Qout
// unused).  MODE 1: RK stage, res in place, Qout = Qin + b res.  smem:
// Fp64Smem<N,EPB>::size doubles.  nt: non-temporal res read and stores.
template <int N, int MODE, int EPB, int NT>
__device__ __forceinline__ void stage_nb_body(const DGTables& tb, const double* __restrict__ Qin,
                                              double* __restrict__ Qout, double* __restrict__ RR, double rka,
                                              double rkb, double dt, int first, int e0, int ne, bool nt,
                                              double* smem, int tid) {
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

  for (int x = tid; x < N * N; x += NT) sDh[x] = tb.Dh[x];
  if (tid < N) {
    sLm[tid] = tb.lm[tid];
    sLp[tid] = tb.lp[tid];
    sLiftm[tid] = tb.liftm[tid];
    sLiftp[tid] = tb.liftp[tid];
  }
  double lmr[N], lpr[N];             // l(-1), l(+1) in registers (kernarg tables)
#pragma unroll
  for (int m = 0; m < N; ++m) {
    lmr[m] = tb.lm[m];
    lpr[m] = tb.lp[m];
  }

  // ---- A: this thread's node, residual register, neighbour traces
  const bool nthr = tid < NODES;
  const int el = tid / N3;
  const int t = tid - el * N3;
  const int ni = t % N, nj = (t / N) % N, nk = t / N2;
  const int e = e0 + el;
  const bool act = nthr && el < ne;
  const int64_t gofs = (int64_t)e * N3 + t;
  double q[5], r[5];
  if (act) {
#pragma unroll
    for (int f = 0; f < 5; ++f) q[f] = Qin[f * EN3 + gofs];
  } else {
    q[0] = 1.0; q[1] = 0.0; q[2] = 0.0; q[3] = 0.0; q[4] = 2.5;
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) r[f] = 0.0;
  if (MODE != 0 && act && !first) {
#pragma unroll
    for (int f = 0; f < 5; ++f) r[f] = ld_stream(RR + f * EN3 + gofs, nt);
  }
  if (nthr) {
#pragma unroll
    for (int f = 0; f < 5; ++f) sQ[f * NODES + tid] = q[f];
  }
  double nb[IPT][5];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int it = tid + u * NT;
    const int face = it / FP;
    const int rem = it - face * FP;
    const int fel = rem / N2;
    const int pt = rem - fel * N2;
    const int ee = e0 + fel;
    if (it < NITEM && fel < ne) {
      const int d = face >> 1, side = face & 1;
      const int nbe = neighbour(tb.nx, tb.ny, tb.nz, ee, d, side ? 1 : -1);
      // the neighbour's face on the other side: its -d face for our +d face
      const double* base = Qin + (int64_t)nbe * N3;
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        const double* qn = base + f * EN3;
        double v = 0.0;
#pragma unroll
        for (int m = 0; m < N; ++m) v = fma(side ? lmr[m] : lpr[m], qn[tnode<N>(d, m, pt)], v);
        nb[u][f] = v;
      }
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
  const double rinv = 1.0 / q[0];
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
      for (int f = 0; f < 5; ++f) st_stream(RR + f * EN3 + gofs, acc[f], nt);
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
        st_stream(Qout + f * EN3 + gofs, q[f], nt);
        st_stream(RR + f * EN3 + gofs, r[f], nt);
      }
    }
  }
}

}  // namespace dgdev
