// Batched persistent kernels: many independent periodic meshes of uneven
// size and polynomial degree advanced by one launch per RK stage.
//
// A work list of (mesh, first element) items, one item per block of up to
// EPB consecutive elements of one x-row, is walked by a persistent grid
// (static round robin: item k belongs to block k mod gridDim).  Each item
// runs the same fused
// neighbour-read stage body as the single-mesh kernel (stage_nb.h /
// stage_nb32.h) with the compile-time degree N and elements-per-workgroup
// EPB of its mesh, on a shared-memory buffer sized for the largest (N, EPB)
// variant.  Every variant uses 256 threads.  The state of all meshes
// alternates between two buffers (Qin -> Qout) from launch to launch.

#include "dg_batch.h"
#include "stage_fp32.h"
#include "stage_nb32.h"
#include "stage_fp64.h"
#include "stage_nb.h"

namespace {

constexpr int BNT = 256;

// (N, EPB) variants compiled into the batched kernels.
#define DG_BATCH_VARIANTS(X) \
  X(2, 8) X(2, 16) X(3, 4) X(3, 9) X(4, 2) X(4, 4) X(5, 1) X(5, 2) X(6, 1)

template <int N, int EPB>
constexpr int smax64() { return dgdev::NbSmem<N, EPB>::size; }
template <int N, int EPB>
constexpr int smax32() { return dgdev::Nb32Smem<N, EPB>::bytes; }

constexpr int cmax(int a, int b) { return a > b ? a : b; }
#define DG_SZ64(n, e) smax64<n, e>(),
#define DG_SZ32(n, e) smax32<n, e>(),
constexpr int kSizes64[] = {DG_BATCH_VARIANTS(DG_SZ64) 0};
constexpr int kSizes32[] = {DG_BATCH_VARIANTS(DG_SZ32) 0};
constexpr int arrmax(const int* a, int n) { return n == 0 ? 0 : cmax(a[0], arrmax(a + 1, n - 1)); }
constexpr int kSmem64 = arrmax(kSizes64, sizeof(kSizes64) / sizeof(int));          // doubles
constexpr int kSmem32 = (arrmax(kSizes32, sizeof(kSizes32) / sizeof(int)) + 7) / 8;  // doubles

// How the FP64 variants read their y/z neighbour lines: partner-lane pairs
// at even N, LDS-handed pairs at odd N.  The FP32 variants read one point
// per lane: partner-lane pairs would take their union of registers from
// three waves per SIMD to two.
template <int N>
constexpr int kLines64 = N % 2 == 0 ? dgdev::LINES_DPP : dgdev::LINES_LDS;

template <int MODE, bool F32>
__device__ __forceinline__ void run_item(const DGBatchInst& I, int e0, const double* Qin, double* Qout, double* RR,
                                         double a, double b, int first, double* smem, int tid) {
  // uniform across the workgroup: an SGPR value keeps the dispatch a scalar
  // branch (a divergent switch would overlap every variant's registers)
  const int key = __builtin_amdgcn_readfirstlane(I.N * 64 + I.epb);
  const double* qi = Qin + I.qoff;
  double* qo = Qout ? Qout + I.qoff : nullptr;
  double* rr = RR + I.qoff;
  // items are row-aligned blocks: the last block of a row may be short
  const int x0 = e0 % I.tab.nx;
  const int ne = dgdev::imin(I.epb, I.tab.nx - x0);
#define DG_CASE(n, e)                                                                                                       \
  case n * 64 + e:                                                                                                          \
    if (F32)                                                                                                                \
      dgdev::stage_nb32_body<n, MODE, e, BNT, dgdev::LINES_POINT>(I.tab, qi, qo, rr, a, b, I.dt, first, e0, ne, smem, tid); \
    else                                                                                                                    \
      dgdev::stage_nb_body<n, MODE, e, BNT, kLines64<n>>(I.tab, qi, qo, rr, a, b, I.dt, first, e0, ne, smem, tid);          \
    break;
  switch (key) { DG_BATCH_VARIANTS(DG_CASE) default: break; }
#undef DG_CASE
}

template <int MODE, bool F32>
__global__ void __launch_bounds__(BNT)
k_batch_stage(const DGBatchInst* __restrict__ inst, const int2* __restrict__ items, int nitems, DGBatchSplit split,
              const double* __restrict__ Qin, double* __restrict__ Qout, double* __restrict__ RR, double a,
              double b, int first) {
  __shared__ double smem[F32 ? kSmem32 : kSmem64];
  int k0 = blockIdx.x, kend = nitems, kstep = gridDim.x;
  if (split.xcd) {
    const int x = blockIdx.x & 7;
    k0 = split.bounds[x] + (blockIdx.x >> 3);
    kend = split.bounds[x + 1];
    kstep = gridDim.x >> 3;
  }
  for (int k = k0; k < kend; k += kstep) {
    const int2 w = items[k];
    const int mi = __builtin_amdgcn_readfirstlane(w.x);
    const int e0 = __builtin_amdgcn_readfirstlane(w.y);
    // An opaque copy of the thread index per item: without it the compiler
    // hoists all thread-index arithmetic of the body out of the loop and
    // keeps it live across items (about 45 extra VGPRs).
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    __syncthreads();  // the previous item's shared-memory reads are complete
    run_item<MODE, F32>(inst[mi], e0, Qin, Qout, RR, a, b, first, smem, tid);
  }
}

}  // namespace

int dg_batch_tile_list(int N, int* out, int max) {
  int n = 0;
#define DG_OPT(nn, e) \
  if (nn == N && n < max) out[n++] = e;
  DG_BATCH_VARIANTS(DG_OPT)
#undef DG_OPT
  return n;
}

int dg_batch_launch_stage(const DGBatchLaunch& L, int mode, const double* Qin, double* Qout, double* RR, double a,
                          double b, int first) {
#define DG_L(m, f)                                                                                           \
  hipLaunchKernelGGL((k_batch_stage<m, f>), dim3(L.grid), dim3(BNT), 0, L.stream, L.inst, L.items, L.nitems, \
                     L.split, Qin, Qout, RR, a, b, first)
  if (L.f32) {
    if (mode == 0) DG_L(0, true);
    else DG_L(1, true);
  } else {
    if (mode == 0) DG_L(0, false);
    else DG_L(1, false);
  }
#undef DG_L
  return (int)hipGetLastError();
}

int dg_batch_blocks_per_cu(int f32) {
  int nb = 0;
  hipError_t e = f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_stage<1, true>, BNT, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_stage<1, false>, BNT, 0);
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}
