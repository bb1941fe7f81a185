// Batched kernels: many independent periodic meshes of uneven size and
// polynomial degree advanced together, per RK stage either one launch per
// degree present (k_batch_degree, the default) or one persistent launch
// (k_batch_stage).
//
// A work list of (mesh, first element) items, one item per block of up to
// EPB consecutive elements of one x-row, grouped by degree.  Each item runs
// the same fused neighbour-read stage body as the single-mesh kernel
// (stage_nb.h / stage_nb32.h) with the compile-time degree N and
// elements-per-workgroup EPB of its mesh; every variant uses 256 threads.
//   k_batch_degree<N, EPB>: one workgroup per item of one degree, with that
//     variant's own registers and shared memory.
//   k_batch_stage: a persistent grid walks the whole list (static round
//     robin: item k belongs to block k mod gridDim) through a shared-memory
//     buffer sized for the largest variant; its register allocation is the
//     union of all variants.
// The state of all meshes alternates between two buffers (Qin -> Qout) from
// launch to launch; the launches of one stage read only Qin.

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

// One (N, EPB) variant over its own items, one workgroup per item
// (DG_BATCH_PER_DEGREE): the variant's own register allocation and shared
// memory.  With xcd set, workgroup w takes item xcd_block(w): each XCD a
// contiguous part of the items.
template <int N, int EPB, int MODE, bool F32>
__global__ void __launch_bounds__(BNT)
k_batch_degree(const DGBatchInst* __restrict__ inst, const int2* __restrict__ items, int begin, int xcd,
               const double* __restrict__ Qin, double* __restrict__ Qout, double* __restrict__ RR, double a,
               double b, int first) {
  __shared__ double smem[F32 ? (smax32<N, EPB>() + 7) / 8 : smax64<N, EPB>()];
  const int w = xcd ? dgdev::xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  const int2 it = items[begin + w];
  const int mi = __builtin_amdgcn_readfirstlane(it.x);
  const int e0 = __builtin_amdgcn_readfirstlane(it.y);
  const DGBatchInst& I = inst[mi];
  const double* qi = Qin + I.qoff;
  double* qo = Qout ? Qout + I.qoff : nullptr;
  double* rr = RR + I.qoff;
  const int x0 = e0 % I.tab.nx;
  const int ne = dgdev::imin(EPB, I.tab.nx - x0);
  if (F32)
    dgdev::stage_nb32_body<N, MODE, EPB, BNT, dgdev::LINES_POINT>(I.tab, qi, qo, rr, a, b, I.dt, first, e0, ne, smem,
                                                                  threadIdx.x);
  else
    dgdev::stage_nb_body<N, MODE, EPB, BNT, kLines64<N>>(I.tab, qi, qo, rr, a, b, I.dt, first, e0, ne, smem,
                                                         threadIdx.x);
}

template <int N, int EPB>
void launch_degree(const DGBatchLaunch& L, int mode, const double* Qin, double* Qout, double* RR, double a, double b,
                   int first) {
  const dim3 grid((unsigned)L.vcount[N]), blk(BNT);
  const int begin = L.vbegin[N];
#define DG_LD(m, f)                                                                                               \
  hipLaunchKernelGGL((k_batch_degree<N, EPB, m, f>), grid, blk, 0, L.stream, L.inst, L.items, begin, L.xcd, Qin, \
                     Qout, RR, a, b, first)
  if (L.f32) {
    if (mode == 0) DG_LD(0, true);
    else DG_LD(1, true);
  } else {
    if (mode == 0) DG_LD(0, false);
    else DG_LD(1, false);
  }
#undef DG_LD
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
  if (L.per_degree) {
    // highest degree first (the costliest launch starts first)
    for (int N = DG_MAXN; N >= 1; --N) {
      if (!L.vcount[N]) continue;
      const int key = N * 64 + L.epb[N];
#define DG_CASE(n, e) \
  case n * 64 + e: launch_degree<n, e>(L, mode, Qin, Qout, RR, a, b, first); break;
      switch (key) {
        DG_BATCH_VARIANTS(DG_CASE)
        default: return (int)hipErrorInvalidValue;
      }
#undef DG_CASE
      const int err = (int)hipGetLastError();
      if (err) return err;
    }
    return 0;
  }
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
