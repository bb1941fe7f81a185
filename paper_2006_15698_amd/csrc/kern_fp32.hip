// FP32 matrix-core variant of the fused DG Euler stage kernel for gfx950.
//
// Same algorithm and phases as the FP64 kernel (kern_fp64.hip), with every
// tensor-product contraction carried out in FP32 on deviations from an FP64
// per-element anchor (the element's first node):
//   volume:  sum_a Dh[m][a] F_a = sum_a Dh[m][a] (F_a - F_ref) + rs[m] F_ref,
//            the first sum on v_mfma_f32_16x16x4_f32 with FP32 accumulation
//            (16 one-dimensional lines per instruction, K = N node index,
//            rows = output node index), the second exactly in FP64 with
//            rs[m] = sum_a Dh[m][a];
//   traces:  T = a + sum_m l_m(+-1) (Q_m - a) with the sum in FP32; the face
//            traces travel between launches as FP32 deviations plus the FP64
//            anchor of their element (half the trace bytes of FP64).
// Pointwise fluxes, the Lax-Friedrichs flux, the lift, the mass matrix and
// the RK accumulation stay FP64, as do Q and res in HBM.  Because both sides
// of a face reconstruct a trace from the same FP32 deviation and FP64
// anchor, the face flux is identical on both sides (discrete conservation
// is kept to FP64 rounding).

#include "dg_internal.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int N> struct FCfg;
template <> struct FCfg<2> { static constexpr int EPB = 16; static constexpr int NT = 128; };
template <> struct FCfg<3> { static constexpr int EPB = 9; static constexpr int NT = 256; };
template <> struct FCfg<4> { static constexpr int EPB = 4; static constexpr int NT = 256; };
template <> struct FCfg<5> { static constexpr int EPB = 2; static constexpr int NT = 256; };
template <> struct FCfg<6> { static constexpr int EPB = 1; static constexpr int NT = 256; };
template <> struct FCfg<7> { static constexpr int EPB = 1; static constexpr int NT = 384; };
template <> struct FCfg<8> { static constexpr int EPB = 1; static constexpr int NT = 512; };

template <int N>
__device__ __forceinline__ int fnode(int d, int m, int pt) {
  if (d == 0) return pt * N + m;
  if (d == 1) return (pt / N) * N * N + m * N + (pt % N);
  return m * N * N + pt;
}

__device__ __forceinline__ int fneighbour(const DGTables& tb, int e, int d, int dir) {
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

// Flux column F^D of Eq. (2), all five fields (D static: see lf_flux32).
template <int D>
__device__ __forceinline__ void flux_dd(const double* q, double gm1, double* F) {
  const double rinv = 1.0 / q[0];
  const double pr = gm1 * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) * rinv);
  const double ud = q[1 + D] * rinv;
  F[0] = q[1 + D];
#pragma unroll
  for (int k = 0; k < 3; ++k) F[1 + k] = q[1 + k] * ud + (k == D ? pr : 0.0);
  F[4] = (q[4] + pr) * ud;
}

__device__ __forceinline__ void flux_d(const double* q, int d, double gm1, double* F) {
  if (d == 0) flux_dd<0>(q, gm1, F);
  else if (d == 1) flux_dd<1>(q, gm1, F);
  else flux_dd<2>(q, gm1, F);
}

// Local Lax-Friedrichs flux, FP64 (Section II-B); the direction is a
// template parameter so that no array is indexed at run time.
template <int D>
__device__ __forceinline__ void lf_flux32_d(const double* qm, const double* qp, double gamma, double gm1,
                                            double* out) {
  double fm[5], fp[5];
  flux_dd<D>(qm, gm1, fm);
  flux_dd<D>(qp, gm1, fp);
  const double rm = 1.0 / qm[0], rp = 1.0 / qp[0];
  const double pm = gm1 * (qm[4] - 0.5 * (qm[1] * qm[1] + qm[2] * qm[2] + qm[3] * qm[3]) * rm);
  const double pp = gm1 * (qp[4] - 0.5 * (qp[1] * qp[1] + qp[2] * qp[2] + qp[3] * qp[3]) * rp);
  const double lm = fabs(qm[1 + D] * rm) + sqrt(gamma * pm * rm);
  const double lp = fabs(qp[1 + D] * rp) + sqrt(gamma * pp * rp);
  const double lam = lm >= lp ? lm : lp;
#pragma unroll
  for (int f = 0; f < 5; ++f) out[f] = 0.5 * (fm[f] + fp[f]) - 0.5 * lam * (qp[f] - qm[f]);
}

__device__ __forceinline__ void lf_flux32(const double* qm, const double* qp, int d, double gamma, double gm1,
                                          double* out) {
  if (d == 0) lf_flux32_d<0>(qm, qp, gamma, gm1, out);
  else if (d == 1) lf_flux32_d<1>(qm, qp, gamma, gm1, out);
  else lf_flux32_d<2>(qm, qp, gamma, gm1, out);
}

// FP32 deviation of the trace of one field on face (d, side) at pt, about
// the anchor value a: sum_m l_m (Q_m - a).  Shared by every kernel that
// produces or consumes traces, so both sides of a face round identically.
template <int N>
__device__ __forceinline__ float trace_dev(const double* sq, const float* coef, int d, int pt, double a) {
  float v = 0.0f;
#pragma unroll
  for (int m = 0; m < N; ++m) v = fmaf(coef[m], (float)(sq[fnode<N>(d, m, pt)] - a), v);
  return v;
}

template <int N>
__host__ __device__ inline size_t anchor_offset(int E) {
  // anchors follow the FP32 deviations, 256-byte aligned
  const size_t b = (size_t)30 * N * N * (size_t)E * sizeof(float);
  return (b + 255) & ~(size_t)255;
}

// Traces of the element states in sQ: FP32 deviations and FP64 anchors.
template <int N, int EPB, int NT>
__device__ __forceinline__ void write_traces32(const double (*sQ)[EPB * N * N * N], const float* sLm,
                                               const float* sLp, int e0, int E, float* __restrict__ T,
                                               double* __restrict__ A) {
  constexpr int N2 = N * N, N3 = N2 * N, FP = EPB * N2;
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
    const float* coef = (face & 1) ? sLp : sLm;
    T[(int64_t)(face * 5 + f) * EN2 + (int64_t)ee * N2 + pt] =
        trace_dev<N>(&sQ[f][fel * N3], coef, face >> 1, pt, sQ[f][fel * N3]);
  }
  for (int x = threadIdx.x; x < 5 * EPB; x += NT) {
    const int f = x / EPB, fel = x % EPB;
    if (e0 + fel < E) A[(int64_t)f * E + e0 + fel] = sQ[f][fel * N3];
  }
}

template <int N>
__global__ void __launch_bounds__(FCfg<N>::NT)
k_trace32(DGTables tb, const double* __restrict__ Q, float* __restrict__ T, double* __restrict__ A) {
  constexpr int EPB = FCfg<N>::EPB, NT = FCfg<N>::NT;
  constexpr int N3 = N * N * N, NODES = EPB * N3;
  __shared__ double sQ[DG_NF][NODES];
  __shared__ float sLm[N], sLp[N];
  const int tid = threadIdx.x;
  const int e0 = blockIdx.x * EPB;
  const int64_t EN3 = (int64_t)tb.E * N3;
  if (tid < N) {
    sLm[tid] = tb.lm32[tid];
    sLp[tid] = tb.lp32[tid];
  }
  for (int x = tid; x < NODES; x += NT) {
    if (e0 + x / N3 < tb.E) {
#pragma unroll
      for (int f = 0; f < 5; ++f) sQ[f][x] = Q[f * EN3 + (int64_t)e0 * N3 + x];
    }
  }
  __syncthreads();
  write_traces32<N, EPB, NT>(sQ, sLm, sLp, e0, tb.E, T, A);
}

// MODE 0: R = dQ/dt.  MODE 1: RK stage.  MODE 2: RK stage + traces out.
template <int N, int MODE>
__global__ void __launch_bounds__(FCfg<N>::NT)
k_stage32(DGTables tb, double* __restrict__ Q, double* __restrict__ RR, const float* __restrict__ Tin,
          const double* __restrict__ Ain, float* __restrict__ Tout, double* __restrict__ Aout, double rka,
          double rkb, double dt, int first) {
  constexpr int EPB = FCfg<N>::EPB, NT = FCfg<N>::NT;
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr int NODES = EPB * N3, FP = EPB * N2;
  constexpr int NITEM = 6 * FP;
  constexpr int IPT = (NITEM + NT - 1) / NT;
  constexpr int NW = NT / 64;
  constexpr int LINES = 5 * EPB * N2;       // 1-D lines per direction
  constexpr int GD = (LINES + 15) / 16;     // MFMA groups per direction
  constexpr int GT = 3 * GD;
  constexpr int GPW = (GT + NW - 1) / NW;   // groups per wave
  constexpr int KS = (N + 3) / 4;           // K steps of 4

  __shared__ double sQ[DG_NF][NODES];
  __shared__ float sF[3][DG_NF][NODES];     // flux deviations, then contraction results
  __shared__ double sH[6][DG_NF][FP];
  __shared__ float sDh[N * N];
  __shared__ float sLm[N], sLp[N];
  __shared__ double sLiftm[N], sLiftp[N], sRs[N];

  const int tid = threadIdx.x;
  const int E = tb.E;
  const int64_t EN3 = (int64_t)E * N3, EN2 = (int64_t)E * N2;
  const int e0 = blockIdx.x * EPB;

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
    for (int f = 0; f < 5; ++f) sQ[f][tid] = q[f];
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
      const int nbe = fneighbour(tb, ee, d, side ? 1 : -1);
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
    for (int f = 0; f < 5; ++f) aq[f] = sQ[f][el * N3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double F[5], Fa[5];
      flux_d(q, d, tb.gm1, F);
      flux_d(aq, d, tb.gm1, Fa);
#pragma unroll
      for (int f = 0; f < 5; ++f) sF[d][f][tid] = (float)(F[f] - Fa[f]);
    }
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
        const double a = sQ[f][fel * N3];
        own[f] = a + (double)trace_dev<N>(&sQ[f][fel * N3], coef, d, pt, a);
      }
      double qm[5], qp[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        qm[f] = side ? own[f] : nb[u][f];
        qp[f] = side ? nb[u][f] : own[f];
      }
      lf_flux32(qm, qp, d, tb.gamma, tb.gm1, fs);
#pragma unroll
      for (int f = 0; f < 5; ++f) sH[face][f][fel * N2 + pt] = fs[f];
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
        const float b = (valid && a < N) ? sF[d][lf][lel * N3 + fnode<N>(d, a < N ? a : 0, lpt)] : 0.0f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Areg[ks], b, acc, 0, 0, 0);
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
          if (i < N) sF[d][lf][lel * N3 + fnode<N>(d, i, lpt)] = res[g][rr];
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
    for (int f = 0; f < 5; ++f) aq[f] = sQ[f][el * N3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int m = d == 0 ? ni : (d == 1 ? nj : nk);
      const int pt = d == 0 ? nj + N * nk : (d == 1 ? ni + N * nk : ni + N * nj);
      double Fa[5];
      flux_d(aq, d, tb.gm1, Fa);
      const double sc = tb.sc[d];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        double s = (double)sF[d][f][tid];
        s = fma(sRs[m], Fa[f], s);
        s = fma(sLiftm[m], sH[2 * d][f][el * N2 + pt], s);
        s = fma(-sLiftp[m], sH[2 * d + 1][f][el * N2 + pt], s);
        acc5[f] = fma(sc, s, acc5[f]);
      }
    }
  }
  if (MODE == 0) {
    if (act) {
#pragma unroll
      for (int f = 0; f < 5; ++f) RR[f * EN3 + gofs] = acc5[f];
    }
    return;
  }
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
      for (int f = 0; f < 5; ++f) sQ[f][tid] = q[f];
    }
    __syncthreads();
    write_traces32<N, EPB, NT>(sQ, sLm, sLp, e0, E, Tout, Aout);
  }
}

template <int N>
int trace32_n(const dg_ctx* c, const double* Q, char* buf) {
  constexpr int EPB = FCfg<N>::EPB;
  const unsigned grid = (unsigned)((c->E + EPB - 1) / EPB);
  float* T = (float*)buf;
  double* A = (double*)(buf + anchor_offset<N>((int)c->E));
  hipLaunchKernelGGL(k_trace32<N>, dim3(grid), dim3(FCfg<N>::NT), 0, c->stream, c->tab, Q, T, A);
  return (int)hipGetLastError();
}

template <int N>
int stage32_n(const dg_ctx* c, double* Q, double* RR, const char* tin, char* tout, int mode, double a, double b,
              double dt, int first) {
  constexpr int EPB = FCfg<N>::EPB;
  const unsigned grid = (unsigned)((c->E + EPB - 1) / EPB);
  const dim3 blk(FCfg<N>::NT);
  const size_t ao = anchor_offset<N>((int)c->E);
  const float* Ti = (const float*)tin;
  const double* Ai = (const double*)(tin + ao);
  float* To = tout ? (float*)tout : nullptr;
  double* Ao = tout ? (double*)(tout + ao) : nullptr;
  if (mode == 0)
    hipLaunchKernelGGL((k_stage32<N, 0>), dim3(grid), blk, 0, c->stream, c->tab, Q, RR, Ti, Ai, To, Ao, a, b, dt, first);
  else if (mode == 1)
    hipLaunchKernelGGL((k_stage32<N, 1>), dim3(grid), blk, 0, c->stream, c->tab, Q, RR, Ti, Ai, To, Ao, a, b, dt, first);
  else
    hipLaunchKernelGGL((k_stage32<N, 2>), dim3(grid), blk, 0, c->stream, c->tab, Q, RR, Ti, Ai, To, Ao, a, b, dt, first);
  return (int)hipGetLastError();
}

}  // namespace

bool dg_f32_supported(int N) { return N >= 2 && N <= DG_MAXN; }

#define DG_F32_DISPATCH(N_, CALL)                \
  switch (N_) {                                  \
    case 2: return CALL(2);                      \
    case 3: return CALL(3);                      \
    case 4: return CALL(4);                      \
    case 5: return CALL(5);                      \
    case 6: return CALL(6);                      \
    case 7: return CALL(7);                      \
    case 8: return CALL(8);                      \
    default: return (int)hipErrorInvalidValue;   \
  }

int dg_launch_trace_f32(const dg_ctx* c, const double* Q, char* buf) {
#define CALL(n) trace32_n<n>(c, Q, buf)
  DG_F32_DISPATCH(c->N, CALL)
#undef CALL
}

int dg_launch_rhs_f32(const dg_ctx* c, const double* Q, const char* tin, double* R) {
#define CALL(n) stage32_n<n>(c, const_cast<double*>(Q), R, tin, nullptr, 0, 0.0, 0.0, 0.0, 0)
  DG_F32_DISPATCH(c->N, CALL)
#undef CALL
}

int dg_launch_stage_f32(const dg_ctx* c, double* Q, double* res, const char* tin, char* tout, double a, double b,
                        double dt, int first) {
  const int mode = tout ? 2 : 1;
#define CALL(n) stage32_n<n>(c, Q, res, tin, tout, mode, a, b, dt, first)
  DG_F32_DISPATCH(c->N, CALL)
#undef CALL
}
