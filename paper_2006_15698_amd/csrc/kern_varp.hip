// Variable polynomial degree per element, on the periodic Cartesian mesh
// with cells optionally refined once into 2 x 2 x 2 children: per RK stage
// one launch for the faces between degrees, one for the hanging faces, then
// one fused RHS / LSERK45 stage launch per (degree, element size) present.
//
// The method of Section II-B on every element with its own degree and size
// (the hp-adaptive setting that Sections I and III name), every face whose
// two sides differ integrated on a mortar: the Gauss-Legendre rule of
// M = max(p, q) + 1 points per tangential direction on the smaller of the
// two faces, both traces evaluated there, the local Lax-Friedrichs flux
// formed once, and the flux integrated against each side's own test
// functions.  With the diagonal collocated mass matrix divided out, the face
// term of a node is the one of Eq. (5) on one element, with the face flux at
// the element's own face nodes replaced by the projection
//     G(t1, t2) = sum_{b1, b2} P[t1][b1] P[t2][b2] F*(b1, b2),
//     P[t][b] = l_t(xi_b) W^M_b / w_t   (times 1/2 on a coarse face's half),
// xi_b the mortar points in the element's own coordinate: x^M_b on a face
// of the mortar's size (F* itself where the element's face nodes are the
// mortar points), (x^M_b + 2h - 1) / 2 on half h of a coarse face; a coarse
// face against four fine ones takes the sum of the four quarters'
// projections.
//
// k_varp_mortar<NLO, NHI, FT>: one launch per degree pair, one wave per face
//   between those degrees (same size): the lower-degree side's trace at its
//   face nodes into LDS, the higher side's trace at its face nodes (the
//   mortar points) in registers (both from the states along the normal
//   lines, or, FT, as the previous stage's launches wrote them into the
//   face-trace buffer), the lower side's trace interpolated to the mortar
//   points, the flux, written for the higher side and projected for the
//   lower side into the face-flux buffer.
// k_varp_hanging (kern_varp_hang.hip): one workgroup per coarse face with
//   hanging faces, one wave per quarter.
// k_varp<N, MODE, TR>: a workgroup owns EPB elements of one degree and size from
// that group's element list (in pencil order; each XCD takes a contiguous
// part), one thread per node:
//   A. the elements' states into LDS (each element's nodes are contiguous);
//      one wave looks up the 6 EPB (face, element) tasks in the face table;
//   B. one point per lane in 64-point slots of one face each: on a
//      conforming face the neighbour's trace interpolated from its state
//      along the normal line (global memory), the own trace from LDS and the
//      flux (the chains of the single-degree kernel); otherwise the
//      projected flux from the buffer;
//   C/D. the volume contraction, lift and RK update of the single-degree
//      neighbour-read kernel, in the same order, so that a mesh of one degree
//      and size gives bitwise the results of that kernel;
//   E. (TR, workgroups with a face that takes its flux from the buffer) the
//      new state into LDS and its traces on those faces into the face-trace
//      buffer, at the faces' flux places, for the next stage's face launches.
// State layout: Q[f * T + off[e] + (k N + j) N + i], T the total node count.

#include "dg_varp.h"
#include "stage_nb.h"

namespace dgdev {
namespace {

template <int N>
struct VCfg {
  // elements per workgroup and threads (one per node, whole waves); the
  // single-degree kernel's tiles from N = 3 on (at most 64 face tasks)
  static constexpr int EPB = N <= 2 ? 8 : (N == 3 ? 9 : (N == 4 ? 4 : (N == 5 ? 2 : 1)));
  static constexpr int NODES = EPB * N * N * N;
  static constexpr int NT = (NODES + 63) / 64 * 64;
  static constexpr int NW = NT / 64;
  static constexpr int FP = EPB * N * N;
  static constexpr int TASKS = 6 * EPB;          // (face, element) pairs
  static constexpr int WPF = (FP + 63) / 64;     // 64-point slots per face
  static constexpr int SMEM = 5 * NODES + 30 * FP + N * N + 2 * N;
  // the new state of a stage that writes its traces: a region of its own
  // (written in the output phase, one barrier before the traces), except
  // at N = 3, where it would cost a workgroup per CU (the state's region is
  // reused after a barrier instead)
  static constexpr bool OWN_NEW = N != 3;
  static constexpr int SMEM_TR = SMEM + (OWN_NEW ? 5 * NODES : 0);
  static_assert(TASKS <= 64, "the face tasks are looked up by one wave");
};

// Flux at point pt of a conforming face (D, SIDE) of an element: the own
// trace from LDS, the neighbour's from its state at qn (global memory),
// the chains of the single-degree kernel.
template <int N, int D, int SIDE>
__device__ __forceinline__ void conforming_flux(const DGTables& tb, const double* own, int ostride,
                                                const double* __restrict__ qn, int64_t T, int pt,
                                                const double* lmr, const double* lpr, double* fs) {
  double nb[5], o[5];
  chunk_trace<N, D, SIDE>(qn, T, 0, pt, lmr, lpr, nb);
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    double v = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) v = fma(SIDE ? lpr[m] : lmr[m], own[f * ostride + tnode<N>(D, m, pt)], v);
    o[f] = v;
  }
  lf_flux_d<D>(SIDE ? o : nb, SIDE ? nb : o, tb.gamma, tb.gm1, fs);
}

// An element's own trace on its face (D, SIDE) at point pt from its state in
// LDS (field stride ostride), written at tr[f N^2].
template <int N, int D, int SIDE>
__device__ __forceinline__ void own_trace(const double* own, int ostride, int pt, const double* lmr,
                                          const double* lpr, double* tr) {
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    double v = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) v = fma(SIDE ? lpr[m] : lmr[m], own[f * ostride + tnode<N>(D, m, pt)], v);
    tr[f * N * N] = v;
  }
}

// One mortar face on one wave, lower side NLO points, higher side NHI = M
// points per direction.  g: this wave's LDS region [5][64] (traces) +
// [5][64] (flux).
template <int NLO, int NHI, bool FT>
__device__ __forceinline__ void mortar_face(const DGTables& tb, const DGVarpTabs* __restrict__ tabs,
                                            const DGVarpMesh& m, const DGVarpFace& F,
                                            const double* __restrict__ Qin, double* g, int lane) {
  constexpr int M = NHI, L2 = NLO * NLO, M2 = M * M;
  const int d = F.d;
  const bool alo = F.code & 1;          // element a (the -d side) has the lower degree
  // a's face is its +1 face, b's its -1 face
  const double* clo = alo ? tabs->lp[NLO] : tabs->lm[NLO];
  const double* chi = alo ? tabs->lm[NHI] : tabs->lp[NHI];
  const int64_t T = m.T;
  double* gL = g;          // [5][64] lower side's trace at its face nodes
  double* gF = g + 320;    // [5][64] flux at the mortar points
  // the interpolation rows of mortar point (b1, b2), loaded while the state
  // lines are in flight
  double r1[NLO], r2[NLO];
  {
    const double* I = tabs->interp[NLO][M];
    const int b1 = lane % M, b2 = (lane < M2 ? lane : 0) / M;
#pragma unroll
    for (int t = 0; t < NLO; ++t) {
      r1[t] = I[b1 * NLO + t];
      r2[t] = I[b2 * NLO + t];
    }
  }
  double th[5];
  if (FT) {
    // both traces as the stage launches wrote them, at the sides' flux places
    const double* tl = m.tbuf + (alo ? F.sa : F.sb);
    const double* tt = m.tbuf + (alo ? F.sb : F.sa);
    if (lane < L2) {
#pragma unroll
      for (int f = 0; f < 5; ++f) gL[f * 64 + lane] = tl[f * L2 + lane];
    }
    if (lane < M2) {
#pragma unroll
      for (int f = 0; f < 5; ++f) th[f] = tt[f * M2 + lane];
    }
  } else {
    if (lane < L2) {
      const double* q = Qin + (alo ? F.oa : F.ob);
      const int a = lane % NLO, b = lane / NLO;
      double w[5][NLO];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
#pragma unroll
        for (int k = 0; k < NLO; ++k) w[f][k] = q[f * T + rt_node<NLO>(d, k, a, b)];
      }
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < NLO; ++k) v = fma(clo[k], w[f][k], v);
        gL[f * 64 + lane] = v;
      }
    }
    if (lane < M2) {
      const double* q = Qin + (alo ? F.ob : F.oa);
      const int a = lane % M, b = lane / M;
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        double w[M];
#pragma unroll
        for (int k = 0; k < M; ++k) w[k] = q[f * T + rt_node<M>(d, k, a, b)];
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) v = fma(chi[k], w[k], v);
        th[f] = v;
      }
    }
  }
  __syncwarp();
  if (lane < M2) {
    double tl[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      double acc = 0.0;
#pragma unroll
      for (int t2 = 0; t2 < NLO; ++t2) {
        double s = 0.0;
#pragma unroll
        for (int t1 = 0; t1 < NLO; ++t1) s = fma(r1[t1], gL[f * 64 + t1 + NLO * t2], s);
        acc = fma(r2[t2], s, acc);
      }
      tl[f] = acc;
    }
    double fs[5];
    lf_flux(alo ? tl : th, alo ? th : tl, d, tb.gamma, tb.gm1, fs);
    double* hhi = m.fbuf + (alo ? F.sb : F.sa);
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      hhi[f * M2 + lane] = fs[f];
      gF[f * 64 + lane] = fs[f];
    }
  }
  __syncwarp();
  if (lane < L2) {
    const double* P = tabs->proj[NLO][M];
    const int t1 = lane % NLO, t2 = lane / NLO;
    double p1[M], p2[M];
#pragma unroll
    for (int b = 0; b < M; ++b) {
      p1[b] = P[t1 * M + b];
      p2[b] = P[t2 * M + b];
    }
    double* hlo = m.fbuf + (alo ? F.sa : F.sb);
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      double acc = 0.0;
#pragma unroll
      for (int b2 = 0; b2 < M; ++b2) {
        double s = 0.0;
#pragma unroll
        for (int b1 = 0; b1 < M; ++b1) s = fma(p1[b1], gF[f * 64 + b1 + M * b2], s);
        acc = fma(p2[b2], s, acc);
      }
      hlo[f * L2 + lane] = acc;
    }
  }
}

constexpr int kMortarWaves = 4;

// One launch per degree pair present (the faces sorted by pair, faces
// [begin, begin + count) of the pair), so that each pair's kernel has its
// own register count: 82-128 VGPRs for the pairs up to (5, 6) against 138
// for one kernel holding every pair.
template <int NLO, int NHI, bool FT>
__global__ void __launch_bounds__(64 * kMortarWaves) k_varp_mortar(const DGTables tb, const DGVarpMesh m,
                                                                    const double* __restrict__ Qin, int begin,
                                                                    int count) {
  __shared__ double sg[kMortarWaves][640];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int fi = blockIdx.x * kMortarWaves + wave;
  if (fi >= count) return;   // whole waves: no workgroup barrier below
  const DGVarpFace F = m.faces[begin + fi];
  mortar_face<NLO, NHI, FT>(tb, m.tabs, m, F, Qin, sg[wave], lane);
}

template <int NLO, int NHI>
int launch_mortar(hipStream_t stream, const DGTables& tb, const DGVarpMesh& m, const double* Qin, int begin,
                  int count, bool ft) {
  const unsigned grid = (unsigned)((count + kMortarWaves - 1) / kMortarWaves);
  if (ft)
    hipLaunchKernelGGL((k_varp_mortar<NLO, NHI, true>), dim3(grid), dim3(64 * kMortarWaves), 0, stream, tb, m, Qin,
                       begin, count);
  else
    hipLaunchKernelGGL((k_varp_mortar<NLO, NHI, false>), dim3(grid), dim3(64 * kMortarWaves), 0, stream, tb, m, Qin,
                       begin, count);
  return (int)hipGetLastError();
}

template <int N, int MODE, bool TR>
__global__ void __launch_bounds__(VCfg<N>::NT) __attribute__((amdgpu_waves_per_eu(N == 4 || N == 6 ? 4 : 1, 8))) k_varp(const DGTables tb, const DGVarpMesh mesh, int first,
                                                      int count, const double* __restrict__ Qin,
                                                      double* __restrict__ Qout, double* __restrict__ RR,
                                                      double rka, double rkb, double dt) {
  using C = VCfg<N>;
  constexpr int N2 = N * N, N3 = N2 * N, EPB = C::EPB, NODES = C::NODES, FP = C::FP;
  constexpr int TASKS = C::TASKS, WPF = C::WPF, NW = C::NW;
  __shared__ double smem[TR ? C::SMEM_TR : C::SMEM];
  __shared__ long long sSrc[TASKS];   // the place the face table names
  __shared__ int sKind[TASKS];        // DG_FACE_*
  __shared__ int sAny;                // a task of this block takes its flux from fbuf
  double* sQ = smem;               // [5][NODES] own states; reused as sF in C
  double* sF = smem;
  double* sH = sQ + 5 * NODES;     // [6][5][FP] face flux at the own face nodes
  double* sDh = sH + 30 * FP;      // [N][N]
  double* sLiftm = sDh + N2;
  double* sLiftp = sLiftm + N;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  // each XCD takes a contiguous part of the list (workgroups are dealt to
  // the 8 XCDs round robin)
  const int blk0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
  const int ne = count - blk0 < EPB ? count - blk0 : EPB;
  const int64_t T = mesh.T;

  // ---- A: own states (threads past the block's nodes read element 0's
  //      first node), the face tasks, the 1-D tables
  const int el = tid / N3;
  const int t = tid - el * N3;
  const bool act = tid < NODES && el < ne;
  const int eo = mesh.list[first + blk0 + (act ? el : 0)];
  const int64_t gofs = mesh.off[eo] + (act ? t : 0);
  double q[5], r[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) q[f] = Qin[f * T + gofs];
  if (wave == 0 && lane < TASKS) {
    // task = face * EPB + element
    const int face = lane / EPB, fel = lane - face * EPB;
    long long src = 0;
    int kind = DG_FACE_CONFORMING;
    if (fel < ne) {
      const int e = mesh.list[first + blk0 + fel];
      const long long fr = mesh.face[(int64_t)e * 6 + face];
      kind = (int)(fr & 3);
      src = fr >> 2;
    }
    sSrc[lane] = src;
    sKind[lane] = kind;
    if (TR) {
      const unsigned long long any = __ballot(kind == DG_FACE_MORTAR);
      if (lane == 0) sAny = any != 0ull;
    }
  }
  if (act) {
#pragma unroll
    for (int f = 0; f < 5; ++f) sQ[f * NODES + tid] = q[f];
  }
  // the 1-D tables by selects over uniform kernarg reads (a per-thread index
  // into the argument would copy it to private memory)
  if (tid < N2) {
    double v = 0.0;
#pragma unroll
    for (int x = 0; x < N2; ++x) v = tid == x ? tb.Dh[x] : v;
    sDh[tid] = v;
  }
  if (tid < N) {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      a = tid == m ? tb.liftm[m] : a;
      b = tid == m ? tb.liftp[m] : b;
    }
    sLiftm[tid] = a;
    sLiftp[tid] = b;
  }
  double lmr[N], lpr[N];
#pragma unroll
  for (int m = 0; m < N; ++m) {
    lmr[m] = tb.lm[m];
    lpr[m] = tb.lp[m];
  }
  __syncthreads();

  // ---- B: face points, 64-point slots of one face each (the face is
  //      uniform over a wave)
  for (int s = wave; s < 6 * WPF; s += NW) {
    const int face = s / WPF;
    const int i = (s - face * WPF) * 64 + lane;
    const int fel = i / N2, pt = i - fel * N2;
    if (i < FP && fel < ne) {
      const int task = face * EPB + fel;
      double fs[5];
      if (sKind[task] == DG_FACE_MORTAR) {
        const double* h = mesh.fbuf + sSrc[task];
#pragma unroll
        for (int f = 0; f < 5; ++f) fs[f] = h[f * N2 + pt];
      } else {
        const double* qn = Qin + sSrc[task];
        const double* own = sQ + fel * N3;
        switch (face) {
          case 0: conforming_flux<N, 0, 0>(tb, own, NODES, qn, T, pt, lmr, lpr, fs); break;
          case 1: conforming_flux<N, 0, 1>(tb, own, NODES, qn, T, pt, lmr, lpr, fs); break;
          case 2: conforming_flux<N, 1, 0>(tb, own, NODES, qn, T, pt, lmr, lpr, fs); break;
          case 3: conforming_flux<N, 1, 1>(tb, own, NODES, qn, T, pt, lmr, lpr, fs); break;
          case 4: conforming_flux<N, 2, 0>(tb, own, NODES, qn, T, pt, lmr, lpr, fs); break;
          default: conforming_flux<N, 2, 1>(tb, own, NODES, qn, T, pt, lmr, lpr, fs); break;
        }
      }
#pragma unroll
      for (int f = 0; f < 5; ++f) sH[(face * 5 + f) * FP + i] = fs[f];
    }
  }
  __syncthreads();   // sH complete; sQ is free for sF

  if (MODE == 1) {
#pragma unroll
    for (int f = 0; f < 5; ++f) r[f] = RR[f * T + gofs];
  } else {
#pragma unroll
    for (int f = 0; f < 5; ++f) r[f] = 0.0;
  }
  // ---- C: volume contraction + lift, one direction at a time
  const bool nthr = tid < NODES;
  const int ni = t % N, nj = (t / N) % N, nk = t / N2;
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
      for (int f = 0; f < 5; ++f) RR[f * T + gofs] = acc[f];
    }
  } else {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      r[f] = MODE == 2 ? dt * acc[f] : fma(rka, r[f], dt * acc[f]);
      q[f] = fma(rkb, r[f], q[f]);
    }
    if (act) {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        Qout[f * T + gofs] = q[f];
        RR[f * T + gofs] = r[f];
      }
    }
    // ---- E: the new state's traces on the faces that take their flux from
    //      fbuf, for the next stage's face launches (the same chain as the
    //      face kernels' traces from the state, so the same values)
    if (TR && sAny) {
      double* sN = C::OWN_NEW ? smem + C::SMEM : sQ;
      if (!C::OWN_NEW) __syncthreads();   // the volume phase has read sF
      if (nthr) {
#pragma unroll
        for (int f = 0; f < 5; ++f) sN[f * NODES + tid] = q[f];
      }
      __syncthreads();
      for (int s = wave; s < 6 * WPF; s += NW) {
        const int face = s / WPF;
        const int i = (s - face * WPF) * 64 + lane;
        const int fel = i / N2, pt = i - fel * N2;
        if (i < FP && fel < ne && sKind[face * EPB + fel] == DG_FACE_MORTAR) {
          double* tr = mesh.tbuf + sSrc[face * EPB + fel] + pt;
          const double* own = sN + fel * N3;
          switch (face) {   // uniform over the wave
            case 0: own_trace<N, 0, 0>(own, NODES, pt, lmr, lpr, tr); break;
            case 1: own_trace<N, 0, 1>(own, NODES, pt, lmr, lpr, tr); break;
            case 2: own_trace<N, 1, 0>(own, NODES, pt, lmr, lpr, tr); break;
            case 3: own_trace<N, 1, 1>(own, NODES, pt, lmr, lpr, tr); break;
            case 4: own_trace<N, 2, 0>(own, NODES, pt, lmr, lpr, tr); break;
            default: own_trace<N, 2, 1>(own, NODES, pt, lmr, lpr, tr); break;
          }
        }
      }
    }
  }
}

template <int N>
int launch_varp_n(hipStream_t stream, const DGTables& tb, const DGVarpMesh& m, int first, int count,
                  const double* Qin, double* Qout, double* RR, int mode, double a, double b, double dt, bool tr) {
  if (count <= 0) return 0;
  const unsigned grid = (unsigned)((count + VCfg<N>::EPB - 1) / VCfg<N>::EPB);
  const dim3 blk(VCfg<N>::NT);
#define VARP_LAUNCH(MODE, TR) \
  hipLaunchKernelGGL((k_varp<N, MODE, TR>), dim3(grid), blk, 0, stream, tb, m, first, count, Qin, Qout, RR, a, b, dt)
  if (mode == 0)
    VARP_LAUNCH(0, false);
  else if (mode == 1 && tr)
    VARP_LAUNCH(1, true);
  else if (mode == 1)
    VARP_LAUNCH(1, false);
  else if (tr)
    VARP_LAUNCH(2, true);
  else
    VARP_LAUNCH(2, false);
#undef VARP_LAUNCH
  return (int)hipGetLastError();
}

}  // namespace
}  // namespace dgdev

int dg_varp_epb(int N) {
  using namespace dgdev;
  switch (N) {
    case 1: return VCfg<1>::EPB;
    case 2: return VCfg<2>::EPB;
    case 3: return VCfg<3>::EPB;
    case 4: return VCfg<4>::EPB;
    case 5: return VCfg<5>::EPB;
    case 6: return VCfg<6>::EPB;
    case 7: return VCfg<7>::EPB;
    case 8: return VCfg<8>::EPB;
    default: return 0;
  }
}

int dg_launch_varp(hipStream_t stream, int N, const DGTables& tb, const DGVarpMesh& m, int first, int count,
                   const double* Qin, double* Qout, double* RR, int mode, double a, double b, double dt, bool traces) {
  using namespace dgdev;
#define CALL(n) launch_varp_n<n>(stream, tb, m, first, count, Qin, Qout, RR, mode, a, b, dt, traces && mode != 0)
  switch (N) {
    case 1: return CALL(1);
    case 2: return CALL(2);
    case 3: return CALL(3);
    case 4: return CALL(4);
    case 5: return CALL(5);
    case 6: return CALL(6);
    case 7: return CALL(7);
    case 8: return CALL(8);
    default: return (int)hipErrorInvalidValue;
  }
#undef CALL
}

int dg_launch_varp_mortar(hipStream_t stream, const DGTables& tb, const DGVarpMesh& m, const double* Qin, int lo,
                          int hi, int begin, int count, bool from_traces) {
  using namespace dgdev;
  if (count <= 0) return 0;
#define VARP_PAIR(LO, HI) \
  case (LO) * (DG_VARP_MAXN + 1) + (HI): return launch_mortar<LO, HI>(stream, tb, m, Qin, begin, count, from_traces);
  switch (lo * (DG_VARP_MAXN + 1) + hi) {
    VARP_PAIR(1, 2) VARP_PAIR(1, 3) VARP_PAIR(1, 4) VARP_PAIR(1, 5) VARP_PAIR(1, 6) VARP_PAIR(1, 7) VARP_PAIR(1, 8)
    VARP_PAIR(2, 3) VARP_PAIR(2, 4) VARP_PAIR(2, 5) VARP_PAIR(2, 6) VARP_PAIR(2, 7) VARP_PAIR(2, 8)
    VARP_PAIR(3, 4) VARP_PAIR(3, 5) VARP_PAIR(3, 6) VARP_PAIR(3, 7) VARP_PAIR(3, 8)
    VARP_PAIR(4, 5) VARP_PAIR(4, 6) VARP_PAIR(4, 7) VARP_PAIR(4, 8)
    VARP_PAIR(5, 6) VARP_PAIR(5, 7) VARP_PAIR(5, 8)
    VARP_PAIR(6, 7) VARP_PAIR(6, 8)
    VARP_PAIR(7, 8)
    default: return (int)hipErrorInvalidValue;
  }
#undef VARP_PAIR
}
