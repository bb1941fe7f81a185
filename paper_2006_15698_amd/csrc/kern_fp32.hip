// Single-mesh kernels of the FP32 matrix-core variant: the fused stage with
// the volume contractions on v_mfma_f32_16x16x4_f32, either reading the
// neighbours' states in the same launch (k_stage_nb32, stage_nb32.h, the
// default) or exchanging face traces as FP32 deviations plus FP64 anchors
// between launches (stage_fp32.h).

#include "dg_internal.h"
#include "stage_fp32.h"
#include "stage_nb32.h"
#include "stage_nb.h"

namespace {

template <int N> struct FCfg;
template <> struct FCfg<2> { static constexpr int EPB = 16; static constexpr int NT = 128; };
template <> struct FCfg<3> { static constexpr int EPB = 9; static constexpr int NT = 256; };
template <> struct FCfg<4> { static constexpr int EPB = 4; static constexpr int NT = 256; };
template <> struct FCfg<5> { static constexpr int EPB = 2; static constexpr int NT = 256; };
template <> struct FCfg<6> { static constexpr int EPB = 1; static constexpr int NT = 256; };
template <> struct FCfg<7> { static constexpr int EPB = 1; static constexpr int NT = 384; };
template <> struct FCfg<8> { static constexpr int EPB = 1; static constexpr int NT = 512; };

template <int N>
__global__ void __launch_bounds__(FCfg<N>::NT)
k_trace32(DGTables tb, const double* __restrict__ Q, char* __restrict__ T) {
  constexpr int EPB = FCfg<N>::EPB, NT = FCfg<N>::NT;
  __shared__ double smem[(5 * EPB * N * N * N * 8 + 2 * N * 4 + 7) / 8];
  dgdev::trace_body32<N, EPB, NT>(tb, Q, T, blockIdx.x * EPB, smem, threadIdx.x);
}

template <int N, int MODE>
__global__ void __launch_bounds__(FCfg<N>::NT)
k_stage32(DGTables tb, double* __restrict__ Q, double* __restrict__ RR, const char* __restrict__ Tin,
          char* __restrict__ Tout, double rka, double rkb, double dt, int first) {
  constexpr int EPB = FCfg<N>::EPB, NT = FCfg<N>::NT;
  __shared__ double smem[(dgdev::Fp32Smem<N, EPB>::bytes + 7) / 8];
  dgdev::stage_body32<N, MODE, EPB, NT>(tb, Q, RR, Tin, Tout, rka, rkb, dt, first, blockIdx.x * EPB, smem, threadIdx.x);
}

// At N=5 the bound holds the body to four waves per SIMD (128 registers);
// at N=4 it fits there by itself (120 VGPRs + 4 accumulation registers).
// At N = 2, 4, 6 the y/z neighbour lines are read by partner-lane pairs
// (bitwise the same; N=6 5% faster, N=4 2% beyond the MALL, even at 32^3).
template <int N, int MODE>
__global__ void __launch_bounds__(FCfg<N>::NT) __attribute__((amdgpu_waves_per_eu(N == 5 ? 4 : 1, 8)))
k_stage_nb32(DGTables tb, const double* __restrict__ Qin, double* __restrict__ Qout, double* __restrict__ RR,
             double rka, double rkb, double dt, int first, DGOrder ord) {
  constexpr int EPB = FCfg<N>::EPB, NT = FCfg<N>::NT;
  __shared__ double smem[(dgdev::Nb32Smem<N, EPB>::bytes + 7) / 8];
  int e0, ne;
  dgdev::block_elements<EPB>(tb, ord, blockIdx.x, gridDim.x, e0, ne);
  dgdev::stage_nb32_body<N, MODE, EPB, NT, (N % 2 == 0 && N <= 6) ? dgdev::LINES_DPP : dgdev::LINES_POINT>(
      tb, Qin, Qout, RR, rka, rkb, dt, first, e0, ne, smem, threadIdx.x);
}

template <int N>
int stage_nb32_n(const dg_ctx* c, const double* Qin, double* Qout, double* RR, int mode, double a, double b,
                 double dt, int first) {
  unsigned grid;
  const DGOrder ord = dg_order(c, FCfg<N>::EPB, &grid);
  const dim3 blk(FCfg<N>::NT);
  if (mode == 0)
    hipLaunchKernelGGL((k_stage_nb32<N, 0>), dim3(grid), blk, 0, c->stream, c->tab, Qin, Qout, RR, a, b, dt, first, ord);
  else if (first)
    hipLaunchKernelGGL((k_stage_nb32<N, 2>), dim3(grid), blk, 0, c->stream, c->tab, Qin, Qout, RR, a, b, dt, first, ord);
  else
    hipLaunchKernelGGL((k_stage_nb32<N, 1>), dim3(grid), blk, 0, c->stream, c->tab, Qin, Qout, RR, a, b, dt, first, ord);
  return (int)hipGetLastError();
}

template <int N>
int trace32_n(const dg_ctx* c, const double* Q, char* buf) {
  constexpr int EPB = FCfg<N>::EPB;
  const unsigned grid = (unsigned)((c->E + EPB - 1) / EPB);
  hipLaunchKernelGGL(k_trace32<N>, dim3(grid), dim3(FCfg<N>::NT), 0, c->stream, c->tab, Q, buf);
  return (int)hipGetLastError();
}

template <int N>
int stage32_n(const dg_ctx* c, double* Q, double* RR, const char* tin, char* tout, int mode, double a, double b,
              double dt, int first) {
  constexpr int EPB = FCfg<N>::EPB;
  const unsigned grid = (unsigned)((c->E + EPB - 1) / EPB);
  const dim3 blk(FCfg<N>::NT);
  if (mode == 0)
    hipLaunchKernelGGL((k_stage32<N, 0>), dim3(grid), blk, 0, c->stream, c->tab, Q, RR, tin, tout, a, b, dt, first);
  else if (mode == 1)
    hipLaunchKernelGGL((k_stage32<N, 1>), dim3(grid), blk, 0, c->stream, c->tab, Q, RR, tin, tout, a, b, dt, first);
  else
    hipLaunchKernelGGL((k_stage32<N, 2>), dim3(grid), blk, 0, c->stream, c->tab, Q, RR, tin, tout, a, b, dt, first);
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

int dg_launch_stage_nb_f32(const dg_ctx* c, const double* Qin, double* Qout, double* RR, int mode, double a,
                           double b, double dt, int first) {
#define CALL(n) stage_nb32_n<n>(c, Qin, Qout, RR, mode, a, b, dt, first)
  DG_F32_DISPATCH(c->N, CALL)
#undef CALL
}
