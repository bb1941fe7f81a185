// FP64 kernels of the DG Euler right-hand side and the LSERK45 stage update
// for gfx950.
//
// One workgroup owns EPB consecutive elements and one thread owns one node
// (Section IV: fine-grain parallelism inside an element, one thread per
// mode).  Per workgroup and RK stage:
//   A. load Q (and res) once, coalesced along the SoA layout; stage Q in LDS;
//      prefetch the neighbours' face traces written by the previous launch
//   B. local Lax-Friedrichs flux at every face point of the six faces of
//      every element (own trace interpolated from LDS, Section II-B)
//   C. per direction: pointwise Euler flux F^d (Eq. (2)) into LDS, 1-D
//      sum-factorised volume contraction along the line of the node plus
//      the lift of the two face fluxes on that line (Eq. (5) with the
//      diagonal collocated mass matrix divided out)
//   D. RK axpy in registers, store Q and res, then interpolate the updated Q
//      to the six faces and store those traces for the next stage's
//      neighbours.
// HBM traffic per node and stage: Q and res read and written once (160 B)
// plus the face traces (2 * 6 N^2 * 5 * 8 B per element).

#include "dg_internal.h"

namespace {

template <int N> struct Cfg;
template <> struct Cfg<1> { static constexpr int EPB = 64; static constexpr int NT = 64; };
template <> struct Cfg<2> { static constexpr int EPB = 16; static constexpr int NT = 128; };
template <> struct Cfg<3> { static constexpr int EPB = 9; static constexpr int NT = 256; };
template <> struct Cfg<4> { static constexpr int EPB = 4; static constexpr int NT = 256; };
template <> struct Cfg<5> { static constexpr int EPB = 2; static constexpr int NT = 256; };
template <> struct Cfg<6> { static constexpr int EPB = 1; static constexpr int NT = 256; };
template <> struct Cfg<7> { static constexpr int EPB = 1; static constexpr int NT = 384; };
template <> struct Cfg<8> { static constexpr int EPB = 1; static constexpr int NT = 512; };

// Node index inside an element of the point with index m along direction d
// and tangential index pt = a + N b (lower tangential axis fastest).
template <int N>
__device__ __forceinline__ int tnode(int d, int m, int pt) {
  if (d == 0) return pt * N + m;                          // i = m, j = a, k = b
  if (d == 1) return (pt / N) * N * N + m * N + (pt % N); // j = m, i = a, k = b
  return m * N * N + pt;                                   // k = m, i = a, j = b
}

// Periodic neighbour of element e one step along direction d (dir = +-1).
__device__ __forceinline__ int neighbour(const DGTables& tb, int e, int d, int dir) {
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

// Local Lax-Friedrichs flux across a face with normal +e_D (Section II-B):
// F* = (F^D(qm) + F^D(qp))/2 - lambda/2 (qp - qm),
// lambda = max(|u_D-| + c-, |u_D+| + c+).  Ties pick the - side.  The
// direction is a template parameter so that every array index is static
// (a runtime index would force qm/qp into scratch memory).
template <int D>
__device__ __forceinline__ void lf_flux_d(const double* qm, const double* qp, double gamma, double gm1,
                                          double* out) {
  const double rm = 1.0 / qm[0];
  const double rp = 1.0 / qp[0];
  const double unm = qm[1 + D] * rm;
  const double unp = qp[1 + D] * rp;
  const double pm = gm1 * (qm[4] - 0.5 * (qm[1] * qm[1] + qm[2] * qm[2] + qm[3] * qm[3]) * rm);
  const double pp = gm1 * (qp[4] - 0.5 * (qp[1] * qp[1] + qp[2] * qp[2] + qp[3] * qp[3]) * rp);
  const double lm = fabs(unm) + sqrt(gamma * pm * rm);
  const double lp = fabs(unp) + sqrt(gamma * pp * rp);
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

// Phase D: traces of the element states held in sQ, written to T.
template <int N>
__device__ __forceinline__ void write_traces(const DGTables& tb, const double (*sQ)[Cfg<N>::EPB * N * N * N],
                                             const double* sLm, const double* sLp, int e0,
                                             double* __restrict__ T) {
  constexpr int EPB = Cfg<N>::EPB, NT = Cfg<N>::NT;
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr int FP = EPB * N2;
  const int E = tb.E;
  const int64_t EN2 = (int64_t)E * N2;
  for (int it = threadIdx.x; it < 30 * FP; it += NT) {
    const int pt = it % N2;
    const int r1 = it / N2;
    const int fel = r1 % EPB;
    const int r2 = r1 / EPB;
    const int f = r2 % 5;
    const int face = r2 / 5;
    const int ee = e0 + fel;
    if (ee >= E) continue;
    const int d = face >> 1;
    const double* coef = (face & 1) ? sLp : sLm;
    const double v = line_trace<N>(&sQ[f][fel * N3], coef, d, pt);
    T[(int64_t)(face * 5 + f) * EN2 + (int64_t)ee * N2 + pt] = v;
  }
}

template <int N>
__global__ void __launch_bounds__(Cfg<N>::NT)
k_trace(DGTables tb, const double* __restrict__ Q, double* __restrict__ T) {
  constexpr int EPB = Cfg<N>::EPB, NT = Cfg<N>::NT;
  constexpr int N3 = N * N * N, NODES = EPB * N3;
  __shared__ double sQ[DG_NF][NODES];
  __shared__ double sLm[N], sLp[N];
  const int tid = threadIdx.x;
  const int e0 = blockIdx.x * EPB;
  const int64_t EN3 = (int64_t)tb.E * N3;
  if (tid < N) {
    sLm[tid] = tb.lm[tid];
    sLp[tid] = tb.lp[tid];
  }
  for (int x = tid; x < NODES; x += NT) {
    const int el = x / N3;
    const int e = e0 + el;
    if (e < tb.E) {
#pragma unroll
      for (int f = 0; f < 5; ++f) sQ[f][x] = Q[f * EN3 + (int64_t)e0 * N3 + x];
    }
  }
  __syncthreads();
  write_traces<N>(tb, sQ, sLm, sLp, e0, T);
}

// MODE 0: R = dQ/dt.  MODE 1: RK stage in place.  MODE 2: RK stage in place
// plus the traces of the updated Q into Tout.
template <int N, int MODE>
__global__ void __launch_bounds__(Cfg<N>::NT)
k_stage(DGTables tb, double* __restrict__ Q, double* __restrict__ RR,
        const double* __restrict__ Tin, double* __restrict__ Tout,
        double rka, double rkb, double dt, int first) {
  constexpr int EPB = Cfg<N>::EPB, NT = Cfg<N>::NT;
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr int NODES = EPB * N3, FP = EPB * N2;
  constexpr int NITEM = 6 * FP;
  constexpr int IPT = (NITEM + NT - 1) / NT;

  __shared__ double sQ[DG_NF][NODES];
  __shared__ double sF[DG_NF][NODES];
  __shared__ double sH[6][DG_NF][FP];
  __shared__ double sDh[N * N];
  __shared__ double sLm[N], sLp[N], sLiftm[N], sLiftp[N];

  const int tid = threadIdx.x;
  const int E = tb.E;
  const int64_t EN3 = (int64_t)E * N3;
  const int64_t EN2 = (int64_t)E * N2;
  const int e0 = blockIdx.x * EPB;

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
    for (int f = 0; f < 5; ++f) sQ[f][tid] = q[f];
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
      const int nbe = neighbour(tb, ee, d, side ? 1 : -1);
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
      for (int f = 0; f < 5; ++f) own[f] = line_trace<N>(&sQ[f][fel * N3], coef, d, pt);
      // select values (not pointers) so that nb and own stay in registers
      double qm[5], qp[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        qm[f] = side ? own[f] : nb[u][f];
        qp[f] = side ? nb[u][f] : own[f];
      }
      lf_flux(qm, qp, d, tb.gamma, tb.gm1, fs);
#pragma unroll
      for (int f = 0; f < 5; ++f) sH[face][f][fel * N2 + pt] = fs[f];
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
      sF[0][tid] = q[1 + d];
      sF[1][tid] = q[1] * ud + (d == 0 ? pr : 0.0);
      sF[2][tid] = q[2] * ud + (d == 1 ? pr : 0.0);
      sF[3][tid] = q[3] * ud + (d == 2 ? pr : 0.0);
      sF[4][tid] = (q[4] + pr) * ud;
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
        for (int a = 0; a < N; ++a) s = fma(sDh[m * N + a], sF[f][el * N3 + tnode<N>(d, a, pt)], s);
        s = fma(lfm, sH[2 * d][f][el * N2 + pt], s);
        s = fma(-lfp, sH[2 * d + 1][f][el * N2 + pt], s);
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
    return;
  }
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
      for (int f = 0; f < 5; ++f) sQ[f][tid] = q[f];
    }
    __syncthreads();
    write_traces<N>(tb, sQ, sLm, sLp, e0, Tout);
  }
}

// ---- reductions -----------------------------------------------------------
constexpr int RED_NT = 256;

template <int N>
__global__ void __launch_bounds__(RED_NT)
k_reduce_partial(DGTables tb, const double* __restrict__ Q, double* __restrict__ part) {
  constexpr int N3 = N * N * N;
  __shared__ double sv[DG_RED_VALS][RED_NT];
  const int64_t total = (int64_t)tb.E * N3;
  double s[6] = {0, 0, 0, 0, 0, 0};
  double mx = 0.0, bad = 0.0;
  const int64_t stride = (int64_t)gridDim.x * RED_NT;
  for (int64_t g = (int64_t)blockIdx.x * RED_NT + threadIdx.x; g < total; g += stride) {
    const int t = (int)(g % N3);
    const int i = t % N, j = (t / N) % N, k = t / (N * N);
    const double wq = tb.J * tb.w[i] * tb.w[j] * tb.w[k];
    double q[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) q[f] = Q[f * total + g];
    const double rinv = 1.0 / q[0];
    const double ke = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) * rinv;
    const double pr = tb.gm1 * (q[4] - ke);
#pragma unroll
    for (int f = 0; f < 5; ++f) s[f] += wq * q[f];
    s[5] += wq * ke;
    bool ok = q[0] > 0.0 && pr > 0.0;
#pragma unroll
    for (int f = 0; f < 5; ++f) ok = ok && isfinite(q[f]);
    if (ok) {
      const double c = sqrt(tb.gamma * pr * rinv);
      const double rate = (fabs(q[1] * rinv) + c) * tb.hinv[0] + (fabs(q[2] * rinv) + c) * tb.hinv[1] +
                          (fabs(q[3] * rinv) + c) * tb.hinv[2];
      mx = rate > mx ? rate : mx;
    } else {
      bad += 1.0;
    }
  }
#pragma unroll
  for (int v = 0; v < 6; ++v) sv[v][threadIdx.x] = s[v];
  sv[6][threadIdx.x] = mx;
  sv[7][threadIdx.x] = bad;
  __syncthreads();
  for (int h = RED_NT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const double a = sv[v][threadIdx.x], b = sv[v][threadIdx.x + h];
        sv[v][threadIdx.x] = v == 6 ? (b > a ? b : a) : a + b;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < DG_RED_VALS) part[blockIdx.x * DG_RED_VALS + threadIdx.x] = sv[threadIdx.x][0];
}

__global__ void __launch_bounds__(RED_NT) k_reduce_final(double* __restrict__ part) {
  __shared__ double sv[DG_RED_VALS][RED_NT];
  double acc[DG_RED_VALS];
#pragma unroll
  for (int v = 0; v < DG_RED_VALS; ++v) acc[v] = 0.0;
  for (int b = threadIdx.x; b < DG_RED_BLOCKS; b += RED_NT) {
#pragma unroll
    for (int v = 0; v < DG_RED_VALS; ++v) {
      const double x = part[b * DG_RED_VALS + v];
      acc[v] = v == 6 ? (x > acc[v] ? x : acc[v]) : acc[v] + x;
    }
  }
#pragma unroll
  for (int v = 0; v < DG_RED_VALS; ++v) sv[v][threadIdx.x] = acc[v];
  __syncthreads();
  for (int h = RED_NT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const double a = sv[v][threadIdx.x], b = sv[v][threadIdx.x + h];
        sv[v][threadIdx.x] = v == 6 ? (b > a ? b : a) : a + b;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < DG_RED_VALS) part[DG_RED_BLOCKS * DG_RED_VALS + threadIdx.x] = sv[threadIdx.x][0];
}

template <int N>
int launch_trace_n(const dg_ctx* c, const double* Q, double* T) {
  constexpr int EPB = Cfg<N>::EPB;
  const unsigned grid = (unsigned)((c->E + EPB - 1) / EPB);
  hipLaunchKernelGGL(k_trace<N>, dim3(grid), dim3(Cfg<N>::NT), 0, c->stream, c->tab, Q, T);
  return (int)hipGetLastError();
}

template <int N>
int launch_stage_n(const dg_ctx* c, double* Q, double* RR, const double* Tin, double* Tout,
                   int mode, double a, double b, double dt, int first) {
  constexpr int EPB = Cfg<N>::EPB;
  const unsigned grid = (unsigned)((c->E + EPB - 1) / EPB);
  const dim3 blk(Cfg<N>::NT);
  if (mode == 0)
    hipLaunchKernelGGL((k_stage<N, 0>), dim3(grid), blk, 0, c->stream, c->tab, Q, RR, Tin, Tout, a, b, dt, first);
  else if (mode == 1)
    hipLaunchKernelGGL((k_stage<N, 1>), dim3(grid), blk, 0, c->stream, c->tab, Q, RR, Tin, Tout, a, b, dt, first);
  else
    hipLaunchKernelGGL((k_stage<N, 2>), dim3(grid), blk, 0, c->stream, c->tab, Q, RR, Tin, Tout, a, b, dt, first);
  return (int)hipGetLastError();
}

template <int N>
int launch_reduce_n(const dg_ctx* c, const double* Q, double* red) {
  hipLaunchKernelGGL(k_reduce_partial<N>, dim3(DG_RED_BLOCKS), dim3(RED_NT), 0, c->stream, c->tab, Q, red);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_NT), 0, c->stream, red);
  return (int)hipGetLastError();
}

}  // namespace

#define DG_DISPATCH_N(N_, CALL)                  \
  switch (N_) {                                  \
    case 1: return CALL(1);                      \
    case 2: return CALL(2);                      \
    case 3: return CALL(3);                      \
    case 4: return CALL(4);                      \
    case 5: return CALL(5);                      \
    case 6: return CALL(6);                      \
    case 7: return CALL(7);                      \
    case 8: return CALL(8);                      \
    default: return (int)hipErrorInvalidValue;   \
  }

int dg_launch_trace(const dg_ctx* c, const double* Q, double* T) {
#define CALL(n) launch_trace_n<n>(c, Q, T)
  DG_DISPATCH_N(c->N, CALL)
#undef CALL
}

int dg_launch_rhs(const dg_ctx* c, const double* Q, const double* Tin, double* R) {
#define CALL(n) launch_stage_n<n>(c, const_cast<double*>(Q), R, Tin, nullptr, 0, 0.0, 0.0, 0.0, 0)
  DG_DISPATCH_N(c->N, CALL)
#undef CALL
}

int dg_launch_stage(const dg_ctx* c, double* Q, double* res, const double* Tin, double* Tout,
                    double a, double b, double dt, int first) {
  const int mode = Tout ? 2 : 1;
#define CALL(n) launch_stage_n<n>(c, Q, res, Tin, Tout, mode, a, b, dt, first)
  DG_DISPATCH_N(c->N, CALL)
#undef CALL
}

int dg_launch_reduce(const dg_ctx* c, const double* Q, double* red) {
#define CALL(n) launch_reduce_n<n>(c, Q, red)
  DG_DISPATCH_N(c->N, CALL)
#undef CALL
}
