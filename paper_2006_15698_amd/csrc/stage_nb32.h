// Device code of the FP32 matrix-core stage with neighbour reads.
//
// The block structure of stage_nb_body (stage_nb.h: EPB consecutive
// elements of one x-row, the left and right x-neighbours staged in LDS,
// y/z-neighbour lines read by waves that each handle one face, the state
// loads issued before the first wait, the residual loaded after the face
// phase) with the arithmetic of the FP32 form
// (stage_fp32.h):
//   traces:  T = a + sum_m l_m(+-1) (Q_m - a), a = the FP64 state at the
//            element's first node, the sum in FP32.  The FP32 deviations
//            (Q - a) of the block and of its x-neighbours are formed once per
//            node when they are staged in LDS; a y/z neighbour's line is
//            rounded the same way from global memory, so both sides of a face
//            see the same bits and the face flux cancels exactly;
//   volume:  sum_a Dh[m][a] (F_a - F_ref) on v_mfma_f32_16x16x4_f32 with
//            FP32 accumulation, plus rs[m] F_ref in FP64;
//   LF flux, lift, mass matrix, RK: FP64; Q and res stay FP64 in HBM.
// Results are bitwise those of the trace-buffer FP32 kernels.
#pragma once

#include "stage_fp32.h"
#include "stage_nb.h"

namespace dgdev {

// Shared-memory footprint (bytes) of stage_nb32_body.
template <int N, int EPB>
struct Nb32Smem {
  static constexpr int N3 = N * N * N;
  static constexpr int NODES = EPB * N3;
  static constexpr int NH = (EPB + 2) * N3;
  static constexpr int FP = EPB * N * N;
  static constexpr int dbl = 5 * (EPB + 2) + 30 * FP + 3 * N;             // anchors, sH, lift/rs tables
  static constexpr int devf = 5 * NH;                                     // FP32 deviations (face phase)
  static constexpr int volf = 10 * NODES;                                 // sF, sV (volume phase)
  static constexpr int flt = (devf > volf ? devf : volf) + N * N + 2 * N; // + Dh, l(+-1)
  static constexpr int bytes = dbl * 8 + flt * 4;
};

// FP32 deviation sum of one field's trace on face (D, SIDE) of a chunk
// element read from global memory: its anchor a is the element's first node.
template <int N, int D, int SIDE>
__device__ __forceinline__ void chunk_trace32(const double* __restrict__ base, int64_t EN3, int fel, int pt,
                                              const float* lmr, const float* lpr, double* out) {
  constexpr int N3 = N * N * N;
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const double* qn = base + f * EN3 + fel * N3;
    const double a = qn[0];
    float v = 0.0f;
#pragma unroll
    for (int m = 0; m < N; ++m) v = fmaf(SIDE ? lmr[m] : lpr[m], (float)(qn[tnode<N>(D, m, pt)] - a), v);
    out[f] = a + (double)v;
  }
}

// chunk_trace32 for even N by partner-lane pairs (as chunk_trace_x2 in
// stage_nb.h): each lane loads the line-node pair of its point and its
// x-neighbour at m = 2j + (pt & 1) and takes the other m from its partner by
// DPP.  Same anchor, conversions and FMA chain as chunk_trace32.  Both lanes
// of a pair must be active.
template <int N, int D, int SIDE>
__device__ __forceinline__ void chunk_trace32_x2(const double* __restrict__ base, int64_t EN3, int fel, int pt,
                                                 const float* lmr, const float* lpr, double* out) {
  static_assert(N % 2 == 0, "pairs of x-adjacent points need an even N");
  constexpr int N3 = N * N * N;
  const int s = pt & 1;
  const int pe = pt - s;
  double2 w[5][N / 2];
  double an[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const double* qn = base + f * EN3 + fel * N3;
    an[f] = qn[0];
#pragma unroll
    for (int j = 0; j < N / 2; ++j)
      __builtin_memcpy(&w[f][j], qn + (s ? tnode<N>(D, 2 * j + 1, pe) : tnode<N>(D, 2 * j, pe)), 16);
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const double a = an[f];
    float v = 0.0f;
#pragma unroll
    for (int j = 0; j < N / 2; ++j) {
      const double px = swap_adjacent(w[f][j].x), py = swap_adjacent(w[f][j].y);
      v = fmaf(SIDE ? lmr[2 * j] : lpr[2 * j], (float)((s ? py : w[f][j].x) - a), v);
      v = fmaf(SIDE ? lmr[2 * j + 1] : lpr[2 * j + 1], (float)((s ? w[f][j].y : px) - a), v);
    }
    out[f] = a + (double)v;
  }
}

// FP32 deviation sum along the line of point pt in direction D of an
// element whose deviations are at `dev` (LDS, field stride NH).
template <int N, int D>
__device__ __forceinline__ float line_dev(const float* dev, const float* coef, int pt) {
  float v = 0.0f;
#pragma unroll
  for (int m = 0; m < N; ++m) v = fmaf(coef[m], dev[tnode<N>(D, m, pt)], v);
  return v;
}

// LF flux at point pt of face (D, SIDE) of the block element in slot `so`;
// the neighbour is the LDS slot `sn` (x-faces) or the registers nbv.
template <int N, int D, int SIDE, bool LDSNB>
__device__ __forceinline__ void face_flux32(const float* sD, const double* sAnc, int so, int sn, const double* nbv,
                                            int NH, int NS, int pt, const float* sLm, const float* sLp,
                                            double gamma, double gm1, double* fs) {
  constexpr int N3 = N * N * N;
  double qm[5], qp[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const double o = sAnc[f * NS + so] + (double)line_dev<N, D>(sD + f * NH + so * N3, SIDE ? sLp : sLm, pt);
    const double n =
        LDSNB ? sAnc[f * NS + sn] + (double)line_dev<N, D>(sD + f * NH + sn * N3, SIDE ? sLm : sLp, pt) : nbv[f];
    qm[f] = SIDE ? o : n;
    qp[f] = SIDE ? n : o;
  }
  lf_flux32_d<D>(qm, qp, gamma, gm1, fs);
}

// Elements [e0, e0 + ne) of one x-row, ne <= EPB.  MODE 0: RR = dQ/dt.
// MODE 1: RK stage (res = RR in place).  MODE 2: the first RK stage (a = 0:
// res written, not read).  NBL: LINES_DPP reads the y/z neighbour lines
// by partner-lane pairs (even N), anything else one point per lane.  smem:
// Nb32Smem<N,EPB>::bytes.
template <int N, int MODE, int EPB, int NT, int NBL>
__device__ __forceinline__ void stage_nb32_body(const DGTables& tb, const double* __restrict__ Qin,
                                                double* __restrict__ Qout, double* __restrict__ RR, double rka,
                                                double rkb, double dt, int first, int e0, int ne, double* smem,
                                                int tid) {
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr int NODES = EPB * N3, FP = EPB * N2, NH = (EPB + 2) * N3, NS = EPB + 2;
  constexpr int NW = NT / 64;
  using S = FaceSlots<N, EPB>;
  constexpr int RND = (S::NS + NW - 1) / NW;
  constexpr int RNDG = (S::NYZ + NW - 1) / NW;
  constexpr int LINES = 5 * EPB * N2;       // 1-D lines per direction
  constexpr int GD = (LINES + 15) / 16;     // matrix-core groups per direction
  constexpr int GPW = (GD + NW - 1) / NW;   // groups per wave and direction
  constexpr int KS = (N + 3) / 4;           // K steps of 4
  using SM = Nb32Smem<N, EPB>;
  static_assert(NODES <= NT, "one thread per node");
  static_assert(NT % 64 == 0, "whole waves");

  double* sAnc = smem;                        // [5][NS] anchors (first node of each slot's element)
  double* sH = sAnc + 5 * NS;                 // [6][5][FP] face fluxes
  double* sLiftm = sH + 30 * FP;
  double* sLiftp = sLiftm + N;
  double* sRs = sLiftp + N;
  float* sD = (float*)(sRs + N);              // [5][NH] FP32 deviations (face phase)
  float* sF = sD;                             // [5][NODES] flux deviations of one direction (volume phase)
  float* sV = sF + 5 * NODES;                 // [5][NODES] their contraction
  float* sDh = sD + (SM::devf > SM::volf ? SM::devf : SM::volf);
  float* sLm = sDh + N * N;
  float* sLp = sLm + N;

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

  float lmr[N], lpr[N];
#pragma unroll
  for (int m = 0; m < N; ++m) {
    lmr[m] = tb.lm32[m];
    lpr[m] = tb.lp32[m];
  }

  // ---- A: every state load before the first wait (see stage_nb_body)
  const bool nthr = tid < NODES;
  const int el = tid / N3;
  const int t = tid - el * N3;
  const int ni = t % N, nj = (t / N) % N, nk = t / N2;
  const bool act = nthr && el < ne;
  const int64_t gofs = (int64_t)e0 * N3 + tid;
  const int64_t lofs = act ? gofs : (int64_t)e0 * N3;
  constexpr int HPT = (2 * N3 + NT - 1) / NT;
  double q[5], r[5], hq[HPT][5];
#pragma unroll
  for (int f = 0; f < 5; ++f) q[f] = Qin[f * EN3 + lofs];
#pragma unroll
  for (int h = 0; h < HPT; ++h) {
    const int xh = tid + h * NT;
    const int x = xh < 2 * N3 ? xh : 0;
    const int right = x >= N3;
    const double* hb = Qin + (int64_t)(right ? exr : exl) * N3 + (x - right * N3);
#pragma unroll
    for (int f = 0; f < 5; ++f) hq[h][f] = hb[f * EN3];
  }
  const int wave = tid >> 6, lane = tid & 63;
  double nb[RNDG][5];
#pragma unroll
  for (int u = 0; u < RNDG; ++u) {
    const int s = wave + u * NW;
    const int i = (s < S::NYZ ? S::chunk(s) : 0) * 64 + lane;
    const int fel = i / N2, pt = i - fel * N2;
    if (s < S::NYZ && i < FP && fel < ne) {
      if constexpr (NBL == LINES_DPP) {
        static_assert(N % 2 == 0, "partner-lane pairs need an even N");
        // (pairs of lanes share fel, and FP is even: both lanes of a pair
        // take this branch or neither)
        switch (S::face(s)) {   // uniform over the wave
          case 2: chunk_trace32_x2<N, 1, 0>(Qin + (int64_t)eym * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
          case 3: chunk_trace32_x2<N, 1, 1>(Qin + (int64_t)eyp * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
          case 4: chunk_trace32_x2<N, 2, 0>(Qin + (int64_t)ezm * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
          default: chunk_trace32_x2<N, 2, 1>(Qin + (int64_t)ezp * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
        }
      } else {
        switch (S::face(s)) {   // uniform over the wave
          case 2: chunk_trace32<N, 1, 0>(Qin + (int64_t)eym * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
          case 3: chunk_trace32<N, 1, 1>(Qin + (int64_t)eyp * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
          case 4: chunk_trace32<N, 2, 0>(Qin + (int64_t)ezm * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
          default: chunk_trace32<N, 2, 1>(Qin + (int64_t)ezp * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
        }
      }
    } else {
      nb[u][0] = 1.0; nb[u][1] = 0.0; nb[u][2] = 0.0; nb[u][3] = 0.0; nb[u][4] = 2.5;
    }
  }
  // tables from uniform (scalar) kernarg reads
  if (tid < N * N) {
    float v = 0.0f;
#pragma unroll
    for (int x = 0; x < N * N; ++x) v = tid == x ? tb.Dh32[x] : v;
    sDh[tid] = v;
  }
  if (tid < N) {
    float a = 0.0f, b = 0.0f;
    double c = 0.0, d = 0.0, e = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      a = tid == m ? tb.lm32[m] : a;
      b = tid == m ? tb.lp32[m] : b;
      c = tid == m ? tb.liftm[m] : c;
      d = tid == m ? tb.liftp[m] : d;
      e = tid == m ? tb.rs[m] : e;
    }
    sLm[tid] = a;
    sLp[tid] = b;
    sLiftm[tid] = c;
    sLiftp[tid] = d;
    sRs[tid] = e;
  }
  // Anchors: each element's first node, written by the thread that holds it
  // (block slots 1..ne, x-neighbours in slots 0 and ne + 1); then every
  // node's FP32 deviation from its element's anchor.
  if (act && t == 0) {
#pragma unroll
    for (int f = 0; f < 5; ++f) sAnc[f * NS + 1 + el] = q[f];
  }
#pragma unroll
  for (int h = 0; h < HPT; ++h) {
    const int x = tid + h * NT;
    const int right = x >= N3;
    if (x < 2 * N3 && x - right * N3 == 0) {
#pragma unroll
      for (int f = 0; f < 5; ++f) sAnc[f * NS + (right ? ne + 1 : 0)] = hq[h][f];
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int f = 0; f < 5; ++f) sD[f * NH + N3 + tid] = (float)(q[f] - sAnc[f * NS + 1 + el]);
  }
#pragma unroll
  for (int h = 0; h < HPT; ++h) {
    const int x = tid + h * NT;
    if (x < 2 * N3) {
      const int right = x >= N3;
      const int slot = right ? ne + 1 : 0;
#pragma unroll
      for (int f = 0; f < 5; ++f) sD[f * NH + slot * N3 + (x - right * N3)] = (float)(hq[h][f] - sAnc[f * NS + slot]);
    }
  }
  __syncthreads();

  // ---- B: Lax-Friedrichs flux at every face point (FP64)
#pragma unroll
  for (int u = 0; u < RND; ++u) {
    const int s = wave + u * NW;
    const int i = (s < S::NS ? S::chunk(s) : 0) * 64 + lane;
    if (s < S::NS && i < FP) {
      const int face = S::face(s);
      const int fel = i / N2, pt = i - fel * N2;
      const int so = fel + 1;
      const double* nbv = nb[u < RNDG ? u : 0];
      const double g = tb.gamma, g1 = tb.gm1;
      double fs[5];
      switch (face) {   // uniform over the wave
        case 0: face_flux32<N, 0, 0, true>(sD, sAnc, so, so - 1, nbv, NH, NS, pt, sLm, sLp, g, g1, fs); break;
        case 1: face_flux32<N, 0, 1, true>(sD, sAnc, so, so + 1, nbv, NH, NS, pt, sLm, sLp, g, g1, fs); break;
        case 2: face_flux32<N, 1, 0, false>(sD, sAnc, so, so, nbv, NH, NS, pt, sLm, sLp, g, g1, fs); break;
        case 3: face_flux32<N, 1, 1, false>(sD, sAnc, so, so, nbv, NH, NS, pt, sLm, sLp, g, g1, fs); break;
        case 4: face_flux32<N, 2, 0, false>(sD, sAnc, so, so, nbv, NH, NS, pt, sLm, sLp, g, g1, fs); break;
        default: face_flux32<N, 2, 1, false>(sD, sAnc, so, so, nbv, NH, NS, pt, sLm, sLp, g, g1, fs); break;
      }
#pragma unroll
      for (int f = 0; f < 5; ++f) sH[(face * 5 + f) * FP + i] = fs[f];
    }
  }
  __syncthreads();   // last reads of sD; sF and sV reuse it

  // the residual, needed only at the end: loaded here (unconditional in
  // MODE 1: with `first` set it is read and ignored)
  if (MODE == 1) {
#pragma unroll
    for (int f = 0; f < 5; ++f) r[f] = RR[f * EN3 + lofs];
  } else {
#pragma unroll
    for (int f = 0; f < 5; ++f) r[f] = 0.0;
  }
  // ---- C: per direction, matrix-core contraction of the flux deviations.
  // v_mfma_f32_16x16x4_f32: A[i][k] from lane (i = l%16, k = l/16),
  // B[k][j] from lane (k = l/16, j = l%16), D[i][j] in lane j = l%16,
  // register r, row i = 4 (l/16) + r.  Rows i = output node index along
  // the line, k = input node index a, columns j = 16 lines.
  const int li = lane & 15, lk = lane >> 4;
  float Areg[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int a = ks * 4 + lk;
    Areg[ks] = (li < N && a < N) ? sDh[li * N + (a < N ? a : 0)] : 0.0f;
  }
  double aq[5];   // this element's anchor (absent points: the block's first element)
#pragma unroll
  for (int f = 0; f < 5; ++f) aq[f] = sAnc[f * NS + 1 + (act ? el : 0)];
  double acc5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double Fa[5];
    if (d == 0) flux_dd<0>(aq, tb.gm1, Fa);
    else if (d == 1) flux_dd<1>(aq, tb.gm1, Fa);
    else flux_dd<2>(aq, tb.gm1, Fa);
    if (nthr) {
      double F[5];
      if (d == 0) flux_dd<0>(q, tb.gm1, F);
      else if (d == 1) flux_dd<1>(q, tb.gm1, F);
      else flux_dd<2>(q, tb.gm1, F);
#pragma unroll
      for (int f = 0; f < 5; ++f) sF[f * NODES + tid] = (float)(F[f] - Fa[f]);
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < GPW; ++g) {
      const int gi = wave + g * NW;
      if (gi < GD) {
        const int line = gi * 16 + li;
        const bool valid = line < LINES;
        const int lf = valid ? line / (EPB * N2) : 0;
        const int r2 = valid ? line - lf * (EPB * N2) : 0;
        const int lel = r2 / N2;
        const int lpt = r2 - lel * N2;
        f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int a = ks * 4 + lk;
          const float bv = (valid && a < N) ? sF[lf * NODES + lel * N3 + tnode<N>(d, a < N ? a : 0, lpt)] : 0.0f;
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Areg[ks], bv, acc, 0, 0, 0);
        }
        if (valid) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int i = 4 * lk + rr;
            if (i < N) sV[lf * NODES + lel * N3 + tnode<N>(d, i, lpt)] = acc[rr];
          }
        }
      }
    }
    __syncthreads();
    if (nthr) {
      const int m = d == 0 ? ni : (d == 1 ? nj : nk);
      const int pt = d == 0 ? nj + N * nk : (d == 1 ? ni + N * nk : ni + N * nj);
      const double sc = tb.sc[d];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        double s = (double)sV[f * NODES + tid];
        s = fma(sRs[m], Fa[f], s);
        s = fma(sLiftm[m], sH[((2 * d) * 5 + f) * FP + el * N2 + pt], s);
        s = fma(-sLiftp[m], sH[((2 * d + 1) * 5 + f) * FP + el * N2 + pt], s);
        acc5[f] = fma(sc, s, acc5[f]);
      }
    }
    if (d < 2) __syncthreads();   // sV reads done before the next direction's sF/sV writes
  }

  // ---- D: output
  if (MODE == 0) {
    if (act) {
#pragma unroll
      for (int f = 0; f < 5; ++f) RR[f * EN3 + gofs] = acc5[f];
    }
  } else {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      r[f] = (MODE == 2 || first) ? dt * acc5[f] : fma(rka, r[f], dt * acc5[f]);
      q[f] = fma(rkb, r[f], q[f]);
    }
    if (act) {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        Qout[f * EN3 + gofs] = q[f];
        RR[f * EN3 + gofs] = r[f];
      }
    }
  }
}

}  // namespace dgdev
