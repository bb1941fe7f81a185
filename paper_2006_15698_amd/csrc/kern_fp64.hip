// FP64 kernels of the DG Euler right-hand side and the LSERK45 stage update
// for gfx950.
//
// Per RK stage one launch does the pointwise flux, the local Lax-Friedrichs
// face flux, the sum-factorised volume contraction and lift, and the RK
// axpy.  Two ways to obtain a neighbour's state on a shared face:
//   k_stage_nb (stage_nb.h, the default): the neighbour's trace is
//     interpolated from its state in the same launch; the state alternates
//     between two buffers (Qin -> Qout).  HBM traffic per node and stage:
//     Q and res read and written once (160 B) plus neighbour reads that
//     miss the caches.
//   k_stage (stage_fp64.h): each launch also writes the face traces of the
//     updated state, which the next launch reads: 160 B plus
//     2 * 6 N^2 * 5 * 8 B per element.
// Both give bitwise the same results.  The tree reductions below give
// integrals, the maximum wave rate and the state check in a fixed order.

#include "dg_internal.h"
#include "stage_fp64.h"
#include "stage_nb.h"

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

template <int N>
__global__ void __launch_bounds__(Cfg<N>::NT)
k_trace(DGTables tb, const double* __restrict__ Q, double* __restrict__ T) {
  constexpr int EPB = Cfg<N>::EPB, NT = Cfg<N>::NT;
  __shared__ double smem[dgdev::TraceSmem<N, EPB>::size];
  dgdev::trace_body<N, EPB, NT>(tb, Q, T, blockIdx.x * EPB, smem, threadIdx.x);
}

// MODE 0: R = dQ/dt.  MODE 1: RK stage in place.  MODE 2: RK stage in place
// plus the traces of the updated Q into Tout.
template <int N, int MODE>
__global__ void __launch_bounds__(Cfg<N>::NT)
k_stage(DGTables tb, double* __restrict__ Q, double* __restrict__ RR,
        const double* __restrict__ Tin, double* __restrict__ Tout,
        double rka, double rkb, double dt, int first) {
  constexpr int EPB = Cfg<N>::EPB, NT = Cfg<N>::NT;
  __shared__ double smem[dgdev::Fp64Smem<N, EPB>::size];
  dgdev::stage_body<N, MODE, EPB, NT>(tb, Q, RR, Tin, Tout, rka, rkb, dt, first, blockIdx.x * EPB, smem, threadIdx.x);
}

// How the single-mesh stage reads its y/z neighbour lines: partner-lane
// pairs at N = 2, 4, 6 (against one point per lane: N=6 10% faster, N=4
// 6% beyond the MALL and even at 32^3, N=2 1-2%) and, on the row-pair
// layout, at N = 5 (2.5% at 40^3 and 48^3); LDS-handed pairs at N = 7,
// where they are 8% faster (at N = 4, 5, 6 and 8 they were even or 2-7%
// slower); one point per lane at N = 3 and 8 (partner-lane pairs take
// N = 8 past 128 registers).
template <int N>
constexpr int kLines = N == 7 ? dgdev::LINES_LDS
                               : ((N % 2 == 0 && N <= 6) || N == 5) ? dgdev::LINES_DPP : dgdev::LINES_POINT;

// Neighbour-read variant: Qin -> Qout (different buffers), no trace buffers;
// element blocks visited in the order `ord`.  At N=4 the bound holds the
// body to 96 VGPRs, so that five workgroups fit on a CU instead of four
// (about 4% faster).
template <int N, int MODE>
__global__ void __launch_bounds__(Cfg<N>::NT) __attribute__((amdgpu_waves_per_eu(N == 4 ? 5 : 1, 8)))
k_stage_nb(DGTables tb, const double* __restrict__ Qin, double* __restrict__ Qout, double* __restrict__ RR,
           double rka, double rkb, double dt, int first, DGOrder ord) {
  constexpr int EPB = Cfg<N>::EPB, NT = Cfg<N>::NT;
  __shared__ double smem[dgdev::NbSmem<N, EPB>::size];
  int e0, ne;
  dgdev::block_elements<EPB>(tb, ord, blockIdx.x, gridDim.x, e0, ne);
  dgdev::stage_nb_body<N, MODE, EPB, NT, kLines<N>>(tb, Qin, Qout, RR, rka, rkb, dt, first, e0, ne, smem, threadIdx.x);
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
int launch_stage_nb_n(const dg_ctx* c, const double* Qin, double* Qout, double* RR, int mode, double a, double b,
                      double dt, int first) {
  unsigned grid;
  const DGOrder ord = dg_order(c, Cfg<N>::EPB, &grid);
  const dim3 blk(Cfg<N>::NT);
  if (mode == 0)
    hipLaunchKernelGGL((k_stage_nb<N, 0>), dim3(grid), blk, 0, c->stream, c->tab, Qin, Qout, RR, a, b, dt, first, ord);
  else if (first)
    hipLaunchKernelGGL((k_stage_nb<N, 2>), dim3(grid), blk, 0, c->stream, c->tab, Qin, Qout, RR, a, b, dt, first, ord);
  else
    hipLaunchKernelGGL((k_stage_nb<N, 1>), dim3(grid), blk, 0, c->stream, c->tab, Qin, Qout, RR, a, b, dt, first, ord);
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

int dg_launch_stage_nb(const dg_ctx* c, const double* Qin, double* Qout, double* RR, int mode, double a, double b,
                       double dt, int first) {
#define CALL(n) launch_stage_nb_n<n>(c, Qin, Qout, RR, mode, a, b, dt, first)
  DG_DISPATCH_N(c->N, CALL)
#undef CALL
}

int dg_launch_reduce(const dg_ctx* c, const double* Q, double* red) {
#define CALL(n) launch_reduce_n<n>(c, Q, red)
  DG_DISPATCH_N(c->N, CALL)
#undef CALL
}
