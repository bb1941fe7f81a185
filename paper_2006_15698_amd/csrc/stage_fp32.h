// Device code of the FP32 matrix-core variant of the fused DG Euler stage,
// shared by the single-mesh kernels (kern_fp32.hip) and the batched
// persistent kernel (kern_batch.hip).
//
// Same algorithm and phases as the FP64 body (stage_fp64.h), with every
// tensor-product contraction carried out in FP32 on deviations from an FP64
// per-element anchor (the element's first node):
//   volume:  sum_a Dh[m][a] F_a = sum_a Dh[m][a] (F_a - F_ref) + rs[m] F_ref,
//            the first sum on v_mfma_f32_16x16x4_f32 with FP32 accumulation
//            (16 one-dimensional lines per instruction, K = input node index,
//            rows = output node index), the second exactly in FP64 with
//            rs[m] = sum_a Dh[m][a];
//   traces:  T = a + sum_m l_m(+-1) (Q_m - a) with the sum in FP32; the face
//            traces travel between launches as FP32 deviations plus the FP64
//            anchor of their element (half the trace bytes of FP64).
// Pointwise fluxes, the Lax-Friedrichs flux, the lift, the mass matrix and
// the RK accumulation stay FP64, as do Q and res in HBM.  Both sides of a
// face rebuild a trace from the same FP32 deviation and FP64 anchor, so the
// face flux is identical on both sides (discrete conservation is kept).
//
// Trace block of one mesh (bytes): FP32 deviations [face][field][E][N^2],
// then, 256-byte aligned, FP64 anchors [field][E].
#pragma once

#include "dg_internal.h"
#include "stage_fp64.h"

namespace dgdev {

typedef float f4 __attribute__((ext_vector_type(4)));

// Flux column F^D of Eq. (2), all five fields (D static: no runtime index).
template <int D>
__device__ __forceinline__ void flux_dd(const double* q, double gm1, double* F) {
  const double rinv = recip(q[0]);
  const double pr = gm1 * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) * rinv);
  const double ud = q[1 + D] * rinv;
  F[0] = q[1 + D];
#pragma unroll
  for (int k = 0; k < 3; ++k) F[1 + k] = q[1 + k] * ud + (k == D ? pr : 0.0);
  F[4] = (q[4] + pr) * ud;
}

// FP32 deviation of the trace of one field on face (d, side) at pt about
// the anchor value a: sum_m l_m (Q_m - a).  Used by every kernel that
// produces or consumes traces, so both sides of a face round identically.
template <int N>
__device__ __forceinline__ float trace_dev(const double* sq, const float* coef, int d, int pt, double a) {
  float v = 0.0f;
#pragma unroll
  for (int m = 0; m < N; ++m) v = fmaf(coef[m], (float)(sq[tnode<N>(d, m, pt)] - a), v);
  return v;
}

// Byte offset of the anchors inside a mesh's trace block.
template <int N>
__host__ __device__ inline size_t anchor_offset(int E) {
  const size_t b = (size_t)30 * N * N * (size_t)E * sizeof(float);
  return (b + 255) & ~(size_t)255;
}

// Shared-memory footprint (bytes) of the FP32-variant stage body.
template <int N, int EPB>
struct Fp32Smem {
  static constexpr int NODES = EPB * N * N * N;
  static constexpr int FP = EPB * N * N;
  static constexpr int dbl = 5 * NODES + 30 * FP + 3 * N;          // sQ, sH, lift/rs tables
  static constexpr int flt = 15 * NODES + N * N + 2 * N;            // sF, Dh, l(+-1)
  static constexpr int bytes = dbl * 8 + flt * 4;
};

template <int N, int EPB, int NT>
__device__ __forceinline__ void write_traces32(const double* sQ, const float* sLm, const float* sLp, int e0, int E,
                                               char* __restrict__ tblock, int tid) {
  constexpr int N2 = N * N, N3 = N2 * N, NODES = EPB * N3, FP = EPB * N2;
  float* T = (float*)tblock;
  double* A = (double*)(tblock + anchor_offset<N>(E));
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
    const float* coef = (face & 1) ? sLp : sLm;
    const double* sq = sQ + f * NODES + fel * N3;
    T[(int64_t)(face * 5 + f) * EN2 + (int64_t)ee * N2 + pt] = trace_dev<N>(sq, coef, face >> 1, pt, sq[0]);
  }
  for (int x = tid; x < 5 * EPB; x += NT) {
    const int f = x / EPB, fel = x % EPB;
    if (e0 + fel < E) A[(int64_t)f * E + e0 + fel] = sQ[f * NODES + fel * N3];
  }
}

template <int N, int EPB, int NT>
__device__ __forceinline__ void trace_body32(const DGTables& tb, const double* __restrict__ Q, char* __restrict__ tblock,
                                             int e0, double* smem, int tid) {
  constexpr int N3 = N * N * N, NODES = EPB * N3;
  double* sQ = smem;
  float* sLm = (float*)(smem + 5 * NODES);
  float* sLp = sLm + N;
  const int E = tb.E;
  const int64_t EN3 = (int64_t)E * N3;
  if (tid < N) {
    sLm[tid] = tb.lm32[tid];
    sLp[tid] = tb.lp32[tid];
  }
  for (int x = tid; x < NODES; x += NT) {
    if (e0 + x / N3 < E) {
#pragma unroll
      for (int f = 0; f < 5; ++f) sQ[f * NODES + x] = Q[f * EN3 + (int64_t)e0 * N3 + x];
    }
  }
  __syncthreads();
  write_traces32<N, EPB, NT>(sQ, sLm, sLp, e0, E, tblock, tid);
}

template <int D>
__device__ __forceinline__ void lf_flux32_d(const double* qm, const double* qp, double gamma, double gm1,
                                            double* out) {
  double fm[5], fp[5];
  flux_dd<D>(qm, gm1, fm);
  flux_dd<D>(qp, gm1, fp);
  const double rm = recip(qm[0]), rp = recip(qp[0]);
  const double pm = gm1 * (qm[4] - 0.5 * (qm[1] * qm[1] + qm[2] * qm[2] + qm[3] * qm[3]) * rm);
  const double pp = gm1 * (qp[4] - 0.5 * (qp[1] * qp[1] + qp[2] * qp[2] + qp[3] * qp[3]) * rp);
  const double lm = fabs(qm[1 + D] * rm) + root(gamma * pm * rm);
  const double lp = fabs(qp[1 + D] * rp) + root(gamma * pp * rp);
  const double lam = lm >= lp ? lm : lp;
#pragma unroll
  for (int f = 0; f < 5; ++f) out[f] = 0.5 * (fm[f] + fp[f]) - 0.5 * lam * (qp[f] - qm[f]);
}

// MODE 0: RR = dQ/dt.  MODE 1: RK stage.  MODE 2: RK stage + traces out.
// smem: Fp32Smem<N,EPB>::bytes.  tin/tout: trace blocks of this mesh.
template <int N, int MODE, int EPB, int NT>
__device__ __forceinline__ void stage_body32(const DGTables& tb, double* __restrict__ Q, double* __restrict__ RR,
                                             const char* __restrict__ tin, char* __restrict__ tout, double rka,
                                             double rkb, double dt, int first, int e0, double* smem, int tid) {
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr int NODES = EPB * N3, FP = EPB * N2;
  constexpr int NITEM = 6 * FP;
  constexpr int IPT = (NITEM + NT - 1) / NT;
  constexpr int NW = NT / 64;
  constexpr int LINES = 5 * EPB * N2;       // 1-D lines per direction
  constexpr int GD = (LINES + 15) / 16;     // matrix-core groups per direction
  constexpr int GT = 3 * GD;
  constexpr int GPW = (GT + NW - 1) / NW;   // groups per wave
  constexpr int KS = (N + 3) / 4;           // K steps of 4
  static_assert(NODES <= NT, "one thread per node");
  static_assert(NT % 64 == 0, "whole waves");

  double* sQ = smem;                          // [5][NODES]
  double* sH = sQ + 5 * NODES;                // [6][5][FP]
  double* sLiftm = sH + 30 * FP;
  double* sLiftp = sLiftm + N;
  double* sRs = sLiftp + N;
  float* sF = (float*)(sRs + N);              // [3][5][NODES]
  float* sDh = sF + 15 * NODES;               // [N][N]
  float* sLm = sDh + N * N;
  float* sLp = sLm + N;

  const float* Tin = (const float*)tin;
  const int E = tb.E;
  const double* Ain = (const double*)(tin + anchor_offset<N>(E));
  const int64_t EN3 = (int64_t)E * N3, EN2 = (int64_t)E * N2;

  for (int x = tid; x < N * N; x += NT) sDh[x] = tb.Dh32[x];
  if (tid < N) {
    sLm[tid] = tb.lm32[tid];
    sLp[tid] = tb.lp32[tid];
    sLiftm[tid] = tb.liftm[tid];
    sLiftp[tid] = tb.liftp[tid];
    sRs[tid] = tb.rs[tid];
  }

  // ---- A: node state, residual register, neighbour traces
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
      for (int f = 0; f < 5; ++f)
        nb[u][f] = Ain[(int64_t)f * E + nbe] + (double)Tin[(int64_t)(oface * 5 + f) * EN2 + (int64_t)nbe * N2 + pt];
    } else {
      nb[u][0] = 1.0; nb[u][1] = 0.0; nb[u][2] = 0.0; nb[u][3] = 0.0; nb[u][4] = 2.5;
    }
  }
  __syncthreads();

  // ---- flux deviations from the element anchor (FP64, rounded to FP32)
  if (nthr) {
    double aq[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) aq[f] = sQ[f * NODES + el * N3];
    double F[5], Fa[5];
    flux_dd<0>(q, tb.gm1, F);
    flux_dd<0>(aq, tb.gm1, Fa);
#pragma unroll
    for (int f = 0; f < 5; ++f) sF[(0 * 5 + f) * NODES + tid] = (float)(F[f] - Fa[f]);
    flux_dd<1>(q, tb.gm1, F);
    flux_dd<1>(aq, tb.gm1, Fa);
#pragma unroll
    for (int f = 0; f < 5; ++f) sF[(1 * 5 + f) * NODES + tid] = (float)(F[f] - Fa[f]);
    flux_dd<2>(q, tb.gm1, F);
    flux_dd<2>(aq, tb.gm1, Fa);
#pragma unroll
    for (int f = 0; f < 5; ++f) sF[(2 * 5 + f) * NODES + tid] = (float)(F[f] - Fa[f]);
  }
  // ---- B: Lax-Friedrichs flux at every face point (FP64)
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int it = tid + u * NT;
    if (it < NITEM) {
      const int face = it / FP;
      const int rem = it - face * FP;
      const int fel = rem / N2;
      const int pt = rem - fel * N2;
      const int d = face >> 1, side = face & 1;
      const float* coef = side ? sLp : sLm;
      double own[5], fs[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        const double* sq = sQ + f * NODES + fel * N3;
        own[f] = sq[0] + (double)trace_dev<N>(sq, coef, d, pt, sq[0]);
      }
      double qm[5], qp[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        qm[f] = side ? own[f] : nb[u][f];
        qp[f] = side ? nb[u][f] : own[f];
      }
      if (d == 0) lf_flux32_d<0>(qm, qp, tb.gamma, tb.gm1, fs);
      else if (d == 1) lf_flux32_d<1>(qm, qp, tb.gamma, tb.gm1, fs);
      else lf_flux32_d<2>(qm, qp, tb.gamma, tb.gm1, fs);
#pragma unroll
      for (int f = 0; f < 5; ++f) sH[(face * 5 + f) * FP + fel * N2 + pt] = fs[f];
    }
  }
  __syncthreads();

  // ---- C: volume contractions on the matrix cores.
  // v_mfma_f32_16x16x4_f32: A[i][k] from lane (i = l%16, k = l/16),
  // B[k][j] from lane (k = l/16, j = l%16), D[i][j] in lane j = l%16,
  // register r, row i = 4 (l/16) + r.  Rows i = output node index along
  // the line, k = input node index a, columns j = 16 lines.
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  float Areg[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int a = ks * 4 + lk;
    Areg[ks] = (li < N && a < N) ? sDh[li * N + (a < N ? a : 0)] : 0.0f;
  }
  f4 res[GPW];
#pragma unroll
  for (int g = 0; g < GPW; ++g) {
    const int gid = wave + g * NW;
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    if (gid < GT) {
      const int d = gid / GD;
      const int line = (gid - d * GD) * 16 + li;
      const bool valid = line < LINES;
      const int lf = valid ? line / (EPB * N2) : 0;
      const int r2 = valid ? line - lf * (EPB * N2) : 0;
      const int lel = r2 / N2;
      const int lpt = r2 - lel * N2;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int a = ks * 4 + lk;
        const float bv = (valid && a < N) ? sF[(d * 5 + lf) * NODES + lel * N3 + tnode<N>(d, a < N ? a : 0, lpt)]
                                          : 0.0f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Areg[ks], bv, acc, 0, 0, 0);
      }
    }
    res[g] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < GPW; ++g) {
    const int gid = wave + g * NW;
    if (gid < GT) {
      const int d = gid / GD;
      const int line = (gid - d * GD) * 16 + li;
      if (line < LINES) {
        const int lf = line / (EPB * N2);
        const int r2 = line - lf * (EPB * N2);
        const int lel = r2 / N2;
        const int lpt = r2 - lel * N2;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int i = 4 * lk + rr;
          if (i < N) sF[(d * 5 + lf) * NODES + lel * N3 + tnode<N>(d, i, lpt)] = res[g][rr];
        }
      }
    }
  }
  __syncthreads();

  // ---- D: assemble in FP64: contraction + exact constant part + lift
  double acc5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (nthr) {
    double aq[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) aq[f] = sQ[f * NODES + el * N3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int m = d == 0 ? ni : (d == 1 ? nj : nk);
      const int pt = d == 0 ? nj + N * nk : (d == 1 ? ni + N * nk : ni + N * nj);
      double Fa[5];
      if (d == 0) flux_dd<0>(aq, tb.gm1, Fa);
      else if (d == 1) flux_dd<1>(aq, tb.gm1, Fa);
      else flux_dd<2>(aq, tb.gm1, Fa);
      const double sc = tb.sc[d];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        double s = (double)sF[(d * 5 + f) * NODES + tid];
        s = fma(sRs[m], Fa[f], s);
        s = fma(sLiftm[m], sH[((2 * d) * 5 + f) * FP + el * N2 + pt], s);
        s = fma(-sLiftp[m], sH[((2 * d + 1) * 5 + f) * FP + el * N2 + pt], s);
        acc5[f] = fma(sc, s, acc5[f]);
      }
    }
  }
  if (MODE == 0) {
    if (act) {
#pragma unroll
      for (int f = 0; f < 5; ++f) RR[f * EN3 + gofs] = acc5[f];
    }
  } else {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      r[f] = first ? dt * acc5[f] : fma(rka, r[f], dt * acc5[f]);
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
      __syncthreads();  // every anchor read of sQ above is complete
      if (nthr) {
#pragma unroll
        for (int f = 0; f < 5; ++f) sQ[f * NODES + tid] = q[f];
      }
      __syncthreads();
      write_traces32<N, EPB, NT>(sQ, sLm, sLp, e0, E, tout, tid);
    }
  }
}

}  // namespace dgdev
