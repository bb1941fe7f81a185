// Variable polynomial degree per element on the periodic Cartesian mesh:
// one fused RHS / LSERK45 stage launch per degree present.
//
// The method of Section II-B on every element with its own degree (the
// hp-adaptive setting that Sections I and III name), faces between elements
// of degrees p and q integrated on a mortar: the Gauss-Legendre rule of
// M = max(p, q) + 1 points per tangential direction, both traces evaluated
// there, the local Lax-Friedrichs flux formed, and the flux integrated
// against the element's own test functions.  With the diagonal collocated
// mass matrix divided out, the face term of a node is the one of Eq. (5) on
// one element, with the face flux at the element's own face nodes replaced
// by the projection
//     G(t1, t2) = sum_{b1, b2} P[t1][b1] P[t2][b2] F*(b1, b2),
//     P[t][b] = l_t(x^M_b) W^M_b / w_t,
// which is the face flux itself where M equals the element's own point count
// (a conforming face, or a neighbour of lower degree).
//
// A workgroup owns EPB elements of one degree from the degree's element
// list, one thread per node:
//   A. the elements' states into LDS (each element's nodes are contiguous);
//   B. face tasks (element, face) in rounds, each task on a group of GS
//      lanes: (1) the neighbour's trace at its own face nodes, read from
//      global memory along its normal lines, and the own trace from LDS;
//      (2) the flux at the mortar points (interpolating a trace of fewer
//      points); (3) the projection back to the own face nodes;
//   C/D. the volume contraction, lift and RK update of the single-degree
//      neighbour-read kernel, in the same order, so that a mesh of one degree
//      gives bitwise the results of that kernel.
// State layout: Q[f * T + off[e] + (k N + j) N + i], T the total node count.

#include "dg_varp.h"
#include "stage_fp64.h"

namespace dgdev {
namespace {

template <int N>
struct VCfg {
  // elements per workgroup and threads (one per node, whole waves)
  static constexpr int EPB = N <= 2 ? 8 : (N == 3 ? 4 : (N == 4 ? 4 : (N == 5 ? 2 : 1)));
  static constexpr int NODES = EPB * N * N * N;
  static constexpr int NT = (NODES + 63) / 64 * 64;
  static constexpr int FP = EPB * N * N;
};

// LDS doubles of the kernel for a face-task group size gs and a mortar
// point stride mq2 (the largest point count squared in the mesh).
template <int N>
__host__ __device__ constexpr int varp_smem(int gs, int mq2) {
  using C = VCfg<N>;
  return 5 * C::NODES + 30 * C::FP + (C::NT / gs) * (5 * N * N + 10 * mq2) + N * N + 2 * N;
}

// Node of a degree-(n-1) element: index m along direction d, tangential
// point (a, b) (lower tangential axis a), as tnode with a runtime n.
__device__ __forceinline__ int rt_node(int n, int d, int m, int a, int b) {
  if (d == 0) return m + n * (a + n * b);
  if (d == 1) return a + n * (m + n * b);
  return a + n * (b + n * m);
}

// sum_{t2 < n} I[b2 n + t2] sum_{t1 < n} I[b1 n + t1] v[t1 + n t2]: a face
// polynomial given at its n x n nodes, evaluated at mortar point (b1, b2).
__device__ __forceinline__ double face_interp(const double* __restrict__ I, int n, int b1, int b2,
                                              const double* v) {
  double acc = 0.0;
  for (int t2 = 0; t2 < n; ++t2) {
    double s = 0.0;
    for (int t1 = 0; t1 < n; ++t1) s = fma(I[b1 * n + t1], v[t1 + n * t2], s);
    acc = fma(I[b2 * n + t2], s, acc);
  }
  return acc;
}

template <int N, int MODE>
__global__ void __launch_bounds__(VCfg<N>::NT) k_varp(const DGTables tb, const DGVarpMesh mesh, int first,
                                                      int count, int gs, int mq2, const double* __restrict__ Qin,
                                                      double* __restrict__ Qout, double* __restrict__ RR,
                                                      double rka, double rkb, double dt) {
  using C = VCfg<N>;
  constexpr int N2 = N * N, N3 = N2 * N, EPB = C::EPB, NODES = C::NODES, FP = C::FP, NT = C::NT;
  extern __shared__ double smem[];
  double* sQ = smem;               // [5][NODES] own states; reused as sF in C
  double* sF = smem;
  double* sH = sQ + 5 * NODES;     // [6][5][FP] face flux at the own face nodes
  double* sDh = sH + 30 * FP;      // [N][N]
  double* sLiftm = sDh + N2;
  double* sLiftp = sLiftm + N;
  double* sG = sLiftp + N;         // per group: own traces [5][N2], neighbour traces [5][mq2], mortar flux [5][mq2]
  const int gstride = 5 * N2 + 10 * mq2;

  const int tid = threadIdx.x;
  const int blk0 = blockIdx.x * EPB;
  const int ne = count - blk0 < EPB ? count - blk0 : EPB;
  const int64_t T = mesh.T;

  // ---- A: own states (threads past the block's nodes read element 0's first node)
  const int el = tid / N3;
  const int t = tid - el * N3;
  const bool act = tid < NODES && el < ne;
  const int eo = mesh.list[first + blk0 + (act ? el : 0)];
  const int64_t gofs = mesh.off[eo] + (act ? t : 0);
  double q[5], r[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) q[f] = Qin[f * T + gofs];
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
  __syncthreads();

  // ---- B: face tasks; task = face * EPB + element, so that the groups of
  //      one wave mostly share a face direction
  const int ng = NT / gs;
  const int g = tid / gs, lg = tid - g * gs;
  double* gO = sG + g * gstride;   // own traces at the own face nodes
  double* gT = gO + 5 * N2;        // neighbour traces at its face nodes
  double* gM = gT + 5 * mq2;       // flux at the mortar points
  const DGVarpTabs* __restrict__ tabs = mesh.tabs;
  const int rounds = (6 * EPB + ng - 1) / ng;
  for (int rd = 0; rd < rounds; ++rd) {
    const int task = rd * ng + g;
    const int face = task / EPB, fel = task - face * EPB;
    const bool live = task < 6 * EPB && fel < ne;
    const int D = face >> 1, side = face & 1;
    int nq = N, M = N;
    if (live) {
      const int e = mesh.list[first + blk0 + fel];
      const int nb = neighbour(mesh.nx, mesh.ny, mesh.nz, e, D, side ? 1 : -1);
      nq = mesh.deg[nb] + 1;
      M = nq > N ? nq : N;
      // (1) the neighbour's trace at its face nodes: its -1 face when ours is +1
      const double* cq = side ? tabs->lm[nq] : tabs->lp[nq];
      const double* qn = Qin + mesh.off[nb];
      for (int k = lg; k < nq * nq; k += gs) {
        const int a = k % nq, b = k / nq;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          double v = 0.0;
          for (int m = 0; m < nq; ++m) v = fma(cq[m], qn[f * T + rt_node(nq, D, m, a, b)], v);
          gT[f * mq2 + k] = v;
        }
      }
      // own trace at the own face nodes (the single-degree kernel's chain)
      const double* own = sQ + fel * N3;
      double co[N];
#pragma unroll
      for (int m = 0; m < N; ++m) co[m] = side ? tb.lp[m] : tb.lm[m];
      for (int k = lg; k < N2; k += gs) {
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          double v = 0.0;
#pragma unroll
          for (int m = 0; m < N; ++m) v = fma(co[m], own[f * NODES + rt_node(N, D, m, k % N, k / N)], v);
          gO[f * N2 + k] = v;
        }
      }
    }
    __syncthreads();
    // (2) flux at the M x M mortar points
    if (live) {
      const double* Io = tabs->interp[N][M];
      const double* In = tabs->interp[nq][M];
      for (int k = lg; k < M * M; k += gs) {
        const int b1 = k % M, b2 = k / M;
        double o[5], n[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          o[f] = M == N ? gO[f * N2 + k] : face_interp(Io, N, b1, b2, gO + f * N2);
          n[f] = M == nq ? gT[f * mq2 + k] : face_interp(In, nq, b1, b2, gT + f * mq2);
        }
        double fs[5];
        lf_flux(side ? o : n, side ? n : o, D, tb.gamma, tb.gm1, fs);
        if (M == N) {
#pragma unroll
          for (int f = 0; f < 5; ++f) sH[(face * 5 + f) * FP + fel * N2 + k] = fs[f];
        } else {
#pragma unroll
          for (int f = 0; f < 5; ++f) gM[f * mq2 + k] = fs[f];
        }
      }
    }
    __syncthreads();
    // (3) projection of a finer mortar's flux onto the own face nodes
    //     (reads only this group's region, which the next round's writes
    //     reach only after its first barrier)
    if (live && M > N) {
      const double* P = tabs->proj[N][M];
      for (int k = lg; k < N2; k += gs) {
        const int t1 = k % N, t2 = k / N;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          double acc = 0.0;
          for (int b2 = 0; b2 < M; ++b2) {
            double s = 0.0;
            for (int b1 = 0; b1 < M; ++b1) s = fma(P[t1 * M + b1], gM[f * mq2 + b1 + M * b2], s);
            acc = fma(P[t2 * M + b2], s, acc);
          }
          sH[(face * 5 + f) * FP + fel * N2 + k] = acc;
        }
      }
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
  }
}

constexpr int kMaxLds = 65536;

// Smallest face-task group (most groups, fewest rounds) whose LDS fits.
template <int N>
int pick_gs(int mq2) {
  constexpr int NT = VCfg<N>::NT;
  for (int gs = 8; gs <= NT; gs *= 2) {
    if (NT % gs) continue;
    if (gs < N * N && gs < 64) continue;   // a conforming face in one pass
    if (varp_smem<N>(gs, mq2) * (int)sizeof(double) <= kMaxLds) return gs;
  }
  return -1;
}

template <int N>
int launch_varp_n(hipStream_t stream, const DGTables& tb, const DGVarpMesh& m, int first, int count,
                  const double* Qin, double* Qout, double* RR, int mode, double a, double b, double dt) {
  if (count <= 0) return 0;
  const int mq2 = m.maxn * m.maxn;
  if (mq2 < N * N || m.maxn > DG_VARP_MAXN) return (int)hipErrorInvalidValue;
  const int gs = pick_gs<N>(mq2);
  if (gs < 0) return (int)hipErrorInvalidConfiguration;
  const size_t lds = (size_t)varp_smem<N>(gs, mq2) * sizeof(double);
  const unsigned grid = (unsigned)((count + VCfg<N>::EPB - 1) / VCfg<N>::EPB);
  const dim3 blk(VCfg<N>::NT);
  if (mode == 0)
    hipLaunchKernelGGL((k_varp<N, 0>), dim3(grid), blk, lds, stream, tb, m, first, count, gs, mq2, Qin, Qout, RR,
                       a, b, dt);
  else if (mode == 1)
    hipLaunchKernelGGL((k_varp<N, 1>), dim3(grid), blk, lds, stream, tb, m, first, count, gs, mq2, Qin, Qout, RR,
                       a, b, dt);
  else
    hipLaunchKernelGGL((k_varp<N, 2>), dim3(grid), blk, lds, stream, tb, m, first, count, gs, mq2, Qin, Qout, RR,
                       a, b, dt);
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
                   const double* Qin, double* Qout, double* RR, int mode, double a, double b, double dt) {
  using namespace dgdev;
#define CALL(n) launch_varp_n<n>(stream, tb, m, first, count, Qin, Qout, RR, mode, a, b, dt)
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
