// Device code of the FP64 DG Euler stage with neighbour reads.
//
// Same arithmetic as stage_body (stage_fp64.h), but the trace of a
// neighbour on a shared face is interpolated from the neighbour's state in
// the same launch (sum over its normal line of l_m(-+1) Q_m, the same FMA
// chain as line_trace) instead of being read from a trace buffer that the
// previous launch wrote.  The state is read from Qin and the updated state
// written to Qout (a different buffer), so no launch reads what it writes.
// Per node and stage the HBM traffic is Q in, res in, Q out, res out
// (160 B) plus whatever neighbour reads miss the caches; there are no trace
// buffers.  Results are bitwise those of stage_body.
//
// A workgroup owns a block of EPB consecutive elements of one x-row.
//   x-faces: the two elements left and right of the block are loaded into
//     LDS next to the block's own elements (coalesced), so every x-face
//     trace, inner or outer, is interpolated from LDS.
//   y- and z-faces: the neighbours of the block are the same EPB elements of
//     an adjacent row, so each face's neighbour chunk has one base address
//     for the whole workgroup; every wave handles points of a single face,
//     so the face's direction and side are compile-time inside the loads.
#pragma once

#include "stage_fp64.h"

namespace dgdev {

__host__ __device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

// How a stage reads its y/z neighbour lines (see stage_nb_body).
enum { LINES_POINT = 0, LINES_LDS = 1, LINES_DPP = 2 };

// Workgroup -> position in the visiting order that gives each XCD a
// contiguous range: workgroups are dispatched round robin over the 8 XCDs,
// so workgroup w runs on XCD w % 8 and is the (w / 8)-th of that XCD.  A
// bijection on [0, nblk) for any nblk.
__host__ __device__ __forceinline__ int xcd_block(int w, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = w & 7, i = w >> 3;
  return x * q + (x < r ? x : r) + i;
}

// Elements [e0, e0 + ne) of workgroup w of nblk under the visiting order o
// (see DGOrder): always ne <= EPB consecutive elements of one x-row.  Every
// value is uniform over the workgroup.
template <int EPB>
__host__ __device__ __forceinline__ void block_elements(const DGTables& tb, const DGOrder& o, int w, int nblk,
                                                        int& e0, int& ne) {
  const int s = o.xcd ? xcd_block(w, nblk) : w;
  const int slab = o.nxb * tb.ny * o.tz;     // blocks of a full z-slab
  const int pz = s / slab;
  int r = s - pz * slab;
  const int tz = imin(o.tz, tb.nz - pz * o.tz);
  const int pen = tb.ny * tz * o.tx;         // blocks of a full pencil of this slab
  const int px = r / pen;
  r -= px * pen;
  const int tx = imin(o.tx, o.nxb - px * o.tx);
  const int y = r / (tz * tx);
  r -= y * (tz * tx);
  const int zz = r / tx;
  const int x0 = (px * o.tx + r - zz * tx) * EPB;
  e0 = ((pz * o.tz + zz) * tb.ny + y) * tb.nx + x0;
  ne = imin(EPB, tb.nx - x0);
}

// Shared-memory footprint (doubles) of stage_nb_body: the state of the
// block and of its two x-neighbours (the flux of one direction reuses it),
// the face fluxes and the 1-D tables.
template <int N, int EPB>
struct NbSmem {
  static constexpr int N3 = N * N * N;
  static constexpr int NH = (EPB + 2) * N3;
  static constexpr int FP = EPB * N * N;
  static constexpr int size = 5 * NH + 30 * FP + N * N + 4 * N;
};

// Face-point slots of a block: a slot is up to 64 points (one wave) of one
// face's EPB N^2 points.  The y- and z-faces (2..5), whose neighbours come
// from global memory, take the first slots; the x-faces (0, 1) the last.
template <int N, int EPB>
struct FaceSlots {
  static constexpr int FP = EPB * N * N;
  static constexpr int WPF = (FP + 63) / 64;   // slots per face
  static constexpr int NS = 6 * WPF;
  static constexpr int NYZ = 4 * WPF;
  __host__ __device__ static constexpr int face(int s) { return s < NYZ ? 2 + s / WPF : (s - NYZ) / WPF; }
  __host__ __device__ static constexpr int chunk(int s) { return s < NYZ ? s % WPF : (s - NYZ) % WPF; }
};

// Trace on our face (D, SIDE) of the neighbour chunk whose first node of
// field 0 is at `base`: element fel of the chunk, tangential point pt.
template <int N, int D, int SIDE>
__device__ __forceinline__ void chunk_trace(const double* __restrict__ base, int64_t EN3, int fel, int pt,
                                            const double* lmr, const double* lpr, double* out) {
  constexpr int N3 = N * N * N;
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const double* qn = base + f * EN3 + fel * N3;
    double v = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) v = fma(SIDE ? lmr[m] : lpr[m], qn[tnode<N>(D, m, pt)], v);
    out[f] = v;
  }
}

// The partner lane's value (lanes 2k and 2k + 1 swap), by DPP.
__device__ __forceinline__ double swap_adjacent(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// chunk_trace for even N, one point per lane: lanes 2k and 2k + 1 hold the
// x-adjacent points pe = pt - s and pe + 1 (s = pt & 1) of one row, whose
// line nodes form a 16-byte-aligned pair at every m (N even).  Each lane
// loads the pair at m = 2j + s and takes its value at the other m of the
// two from its partner, so a lane issues N/2 loads per field instead of N.
// Same FMA chain as chunk_trace, so the traces are bitwise the same.  Both
// lanes of a pair must be active.
template <int N, int D, int SIDE>
__device__ __forceinline__ void chunk_trace_x2(const double* __restrict__ base, int64_t EN3, int fel, int pt,
                                               const double* lmr, const double* lpr, double* out) {
  static_assert(N % 2 == 0, "pairs of x-adjacent points need an even N");
  constexpr int N3 = N * N * N;
  const int s = pt & 1;
  const int pe = pt - s;
  double2 w[5][N / 2];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const double* qn = base + f * EN3 + fel * N3 + tnode<N>(D, 0, pe);
#pragma unroll
    for (int j = 0; j < N / 2; ++j) {
      const int off0 = tnode<N>(D, 2 * j, pe) - tnode<N>(D, 0, pe);
      const int off1 = tnode<N>(D, 2 * j + 1, pe) - tnode<N>(D, 0, pe);
      __builtin_memcpy(&w[f][j], qn + (s ? off1 : off0), 16);
    }
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < N / 2; ++j) {
      const double px = swap_adjacent(w[f][j].x), py = swap_adjacent(w[f][j].y);
      const double a = s ? py : w[f][j].x;   // this point at m = 2j
      const double b = s ? w[f][j].y : px;   // this point at m = 2j + 1
      v = fma(SIDE ? lmr[2 * j] : lpr[2 * j], a, v);
      v = fma(SIDE ? lmr[2 * j + 1] : lpr[2 * j + 1], b, v);
    }
    out[f] = v;
  }
}

// Row-pair lane layout for odd N: each row b of a face chunk element takes
// N + 1 lanes, c = 0..N, so that lanes 2k and 2k + 1 always hold two
// x-adjacent points a = c of one row; lane c = N is a phantom that only
// loads for its partner.  The last pair of a row (c = N - 1, N) reads the
// node pair starting at a = N - 2, so every pair stays inside its row.
template <int N, int EPB>
struct RowPairLane {
  static constexpr int RL = N + 1;
  static constexpr int LANES = EPB * N * RL;
  int fel, b, c;
  bool in;
  __host__ __device__ explicit RowPairLane(int lane) {
    in = lane < LANES;
    fel = lane / (N * RL);
    const int r = lane - fel * (N * RL);
    b = r / RL;
    c = r - b * RL;
  }
  // first point of the node pair this lane loads (its own point is half
  // c & 1 of the pair; the last pair of a row reaches one node past the row,
  // which for the line positions m <= N - 2 that are loaded in pairs is still
  // a node of the element)
  __host__ __device__ int pair_start() const { return (c & ~1) + N * b; }
  // the lane's own point (the phantom lane: the last point of its row)
  __host__ __device__ int own_point() const { return (c < N ? c : N - 1) + N * b; }
};

// chunk_trace for odd N on the row-pair layout: each lane loads the node
// pair of its row pair at m = 2j + s (s = c & 1, j < (N - 1) / 2), sends its
// partner the half that is the partner's point (a select, then one DPP
// swap), and loads its own point at m = N - 1 alone.  Same FMA chain as
// chunk_trace.  Both lanes of a pair must be active.
template <int N, int EPB, int D, int SIDE>
__device__ __forceinline__ void chunk_trace_rp(const double* __restrict__ base, int64_t EN3,
                                               const RowPairLane<N, EPB>& rp, const double* lmr,
                                               const double* lpr, double* out) {
  static_assert(N % 2 == 1, "the row-pair layout is for odd N");
  constexpr int N3 = N * N * N, J = (N - 1) / 2;
  const int s = rp.c & 1;
  const int p0 = rp.pair_start();
  const int po = rp.own_point();
  double2 w[5][J];
  double wl[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const double* qn = base + f * EN3 + rp.fel * N3;
#pragma unroll
    for (int j = 0; j < J; ++j) __builtin_memcpy(&w[f][j], qn + tnode<N>(D, 2 * j + s, p0), 16);
    wl[f] = qn[tnode<N>(D, N - 1, po)];
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      // the pair holds both lanes' points (this lane's is half s): each lane
      // sends the partner's half, so `other` is this lane's point at the
      // partner's m
      const double other = swap_adjacent(s ? w[f][j].x : w[f][j].y);
      v = fma(SIDE ? lmr[2 * j] : lpr[2 * j], s ? other : w[f][j].x, v);
      v = fma(SIDE ? lmr[2 * j + 1] : lpr[2 * j + 1], s ? w[f][j].y : other, v);
    }
    v = fma(SIDE ? lmr[N - 1] : lpr[N - 1], wl[f], v);
    out[f] = v;
  }
}

// Paired neighbour lines.  On a y- or z-face, the line nodes of two face
// points next to each other along x (tangential index a, a + 1 of one row b)
// are next to each other in memory for every m, so one 16-byte load brings
// both (a multi-dword access needs only dword alignment, so a pair may
// start at an odd node).  A lane takes such a pair of points, and the pairs
// of both faces of a direction (the - and + neighbour) share one wave,
// which halves the load instructions of the neighbour lines against one
// point per lane.  Rows of odd length end in a pair that overlaps the
// previous one (a = N-2, N-1).  Used where the pairs of both faces fit one
// wave.
template <int N, int EPB, int NW>
struct PairLines {
  static constexpr int P = (N + 1) / 2;          // pairs per row of a face
  static constexpr int LPF = EPB * N * P;        // lanes per face
  static constexpr bool on = N >= 2 && NW >= 2 && 2 * LPF <= 64;
  static constexpr int FS = NW >= 4 ? 2 : 1;     // field groups: waves per direction
};

// Lane -> pair of face points under PairLines: the face (side 0: the -
// neighbour, 1: the + neighbour), the chunk element fel, the first point pt
// of the pair (the pair is pt, pt + 1 of one row), and whether pt is already
// covered by the row's previous pair.  Lanes from 2 LPF on hold no pair.
template <int N, int EPB>
struct PairLane {
  int side, fel, pt;
  bool dup;
  __host__ __device__ explicit PairLane(int lane) {
    constexpr int P = (N + 1) / 2, LPF = EPB * N * P;
    side = lane >= LPF;
    const int j = lane - side * LPF;
    fel = j / (N * P);
    const int rj = j - fel * (N * P);
    const int b = rj / P, q = rj - b * P;
    const int a0 = 2 * q < N - 2 ? 2 * q : N - 2;
    dup = 2 * q > N - 2;
    pt = a0 + N * b;
  }
};

// Traces of fields [F0, F1) on the faces of direction D (SIDE from the lane)
// for the lane's pair of points, written to the face-flux region sH at
// (face * 5 + f) * FP + fel * N^2 + pt, face = 2 + 2 (D - 1) + side.  The
// FMA chain of each point is that of chunk_trace, so the traces are bitwise
// the same.  Points of absent elements get a valid placeholder state.
template <int N, int EPB, int D, int F0, int F1>
__device__ __forceinline__ void pair_trace(const double* __restrict__ Qin, int64_t EN3, int em, int ep, int ne,
                                           int lane, const double* lmr, const double* lpr, double* sH) {
  constexpr int N2 = N * N, N3 = N2 * N, FP = EPB * N2;
  constexpr int P = (N + 1) / 2, LPF = EPB * N * P;
  if (lane >= 2 * LPF) return;
  const PairLane<N, EPB> pl(lane);
  const int side = pl.side, fel = pl.fel, pt = pl.pt;
  const bool dup = pl.dup;
  double* h = sH + (2 + 2 * (D - 1) + side) * 5 * FP + fel * N2 + pt;
  if (fel < ne) {
    const double* qb = Qin + (int64_t)(side ? ep : em) * N3 + fel * N3 + tnode<N>(D, 0, pt);
    double c[N];
#pragma unroll
    for (int m = 0; m < N; ++m) c[m] = side ? lmr[m] : lpr[m];
    // Up to N = 5: fields in groups of at most 16 loads, each group's loads
    // issued before the first of them is used, held there by a scheduling
    // barrier (left to itself the compiler waits for each load before issuing
    // the next, which costs 10-20% at these degrees).  From N = 6 the
    // compiler's own order is kept: there the registers it saves let one
    // more workgroup onto a CU.
    constexpr bool GROUPED = N <= 5;
    constexpr int G = GROUPED ? 16 / N : 1;
#pragma unroll
    for (int g0 = F0; g0 < F1; g0 += G) {
      double2 w[G][N];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        if (g0 + k < F1) {
          const double* qn = qb + (g0 + k) * EN3;
#pragma unroll
          for (int m = 0; m < N; ++m)
            __builtin_memcpy(&w[k][m], qn + (tnode<N>(D, m, pt) - tnode<N>(D, 0, pt)), 16);
        }
      }
      if constexpr (GROUPED) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < G; ++k) {
        if (g0 + k < F1) {
          double v0 = 0.0, v1 = 0.0;
#pragma unroll
          for (int m = 0; m < N; ++m) {
            v0 = fma(c[m], w[k][m].x, v0);
            v1 = fma(c[m], w[k][m].y, v1);
          }
          if (!dup) h[(g0 + k) * FP] = v0;
          h[(g0 + k) * FP + 1] = v1;
        }
      }
    }
  } else {
#pragma unroll
    for (int f = F0; f < F1; ++f) {
      const double v = f == 0 ? 1.0 : (f == 4 ? 2.5 : 0.0);
      h[f * FP] = v;
      h[f * FP + 1] = v;
    }
  }
}

// Lax-Friedrichs flux at point pt of face (D, SIDE) of the element whose
// state is at `own` (LDS, field stride NH); the neighbour's trace comes
// from LDS (`nbq`, x-faces) or from registers (`nbv`, y- and z-faces).
template <int N, int D, int SIDE, bool LDSNB>
__device__ __forceinline__ void face_flux(const double* own, const double* nbq, const double* nbv, int NH, int pt,
                                          const double* sLm, const double* sLp, double gamma, double gm1,
                                          double* fs) {
  double qm[5], qp[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const double o = line_trace<N>(own + f * NH, SIDE ? sLp : sLm, D, pt);
    const double n = LDSNB ? line_trace<N>(nbq + f * NH, SIDE ? sLm : sLp, D, pt) : nbv[f];
    qm[f] = SIDE ? o : n;
    qp[f] = SIDE ? n : o;
  }
  lf_flux_d<D>(qm, qp, gamma, gm1, fs);
}

// Elements [e0, e0 + ne) of one x-row, ne <= EPB.  MODE 0: RR = dQ/dt (Qout
// unused).  MODE 1: RK stage, res in place (res = a res + dt dQ/dt, or
// dt dQ/dt when `first` is set), Qout = Qin + b res.  MODE 2: the first RK
// stage, whose coefficient a is zero: res = dt dQ/dt is written and the old
// res is not read (40 of the 160 bytes per node).  smem: NbSmem<N,EPB>::size
// doubles.  LINES: how the y/z neighbour lines are read: LINES_POINT one
// point per lane (chunk_trace), LINES_LDS point pairs of both faces of a
// direction per wave with the traces handed over in LDS (PairLines; where
// the configuration allows it, else one point per lane), LINES_DPP point
// pairs of partner lanes (chunk_trace_x2; even N).
template <int N, int MODE, int EPB, int NT, int LINES>
__device__ __forceinline__ void stage_nb_body(const DGTables& tb, const double* __restrict__ Qin,
                                              double* __restrict__ Qout, double* __restrict__ RR, double rka,
                                              double rkb, double dt, int first, int e0, int ne, double* smem,
                                              int tid) {
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr int NODES = EPB * N3, FP = EPB * N2, NH = (EPB + 2) * N3;
  constexpr int NW = NT / 64;
  using S = FaceSlots<N, EPB>;
  constexpr int RND = (S::NS + NW - 1) / NW;     // slot rounds per wave
  constexpr int RNDG = (S::NYZ + NW - 1) / NW;   // rounds that hold y/z slots
  static_assert(NODES <= NT, "one thread per node");
  static_assert(NT % 64 == 0, "whole waves");

  double* sQ = smem;             // [5][NH]: element slot 0 left neighbour, 1..ne own, ne+1 right neighbour
  double* sF = smem;             // [5][NODES]: flux of one direction, reuses sQ after the face phase
  double* sH = sQ + 5 * NH;      // [6][5][FP] face fluxes
  double* sDh = sH + 30 * FP;    // [N][N]
  double* sLm = sDh + N * N;
  double* sLp = sLm + N;
  double* sLiftm = sLp + N;
  double* sLiftp = sLiftm + N;

  const int nx = tb.nx, ny = tb.ny, nz = tb.nz;
  const int64_t EN3 = (int64_t)tb.E * N3;
  // block geometry, uniform: elements x0 .. x0 + ne - 1 of row (ey, ez)
  const int row = e0 / nx;
  const int x0 = e0 - row * nx;
  const int ey = row % ny, ez = row / ny;
  const int plane = nx * ny;
  const int eym = ey == 0 ? e0 + (ny - 1) * nx : e0 - nx;
  const int eyp = ey == ny - 1 ? e0 - (ny - 1) * nx : e0 + nx;
  const int ezm = ez == 0 ? e0 + (nz - 1) * plane : e0 - plane;
  const int ezp = ez == nz - 1 ? e0 - (nz - 1) * plane : e0 + plane;
  const int exl = x0 == 0 ? e0 + nx - 1 : e0 - 1;      // left neighbour of the block
  const int exr = x0 + ne == nx ? e0 - x0 : e0 + ne;    // right neighbour of the block

  double lmr[N], lpr[N];             // l(-1), l(+1) in registers (kernarg tables)
#pragma unroll
  for (int m = 0; m < N; ++m) {
    lmr[m] = tb.lm[m];
    lpr[m] = tb.lp[m];
  }

  // ---- A: the state loads of the block are issued before any is waited
  //         for, in the order of use: own node, the x-neighbours' nodes,
  //         the y/z neighbour traces (loads consumed by their FMA chains;
  //         the load counter completes in order).  The residual, needed
  //         only in D, is loaded at the start of C.
  const bool nthr = tid < NODES;
  const int el = tid / N3;
  const int t = tid - el * N3;
  const int ni = t % N, nj = (t / N) % N, nk = t / N2;
  const bool act = nthr && el < ne;
  const int64_t gofs = (int64_t)e0 * N3 + tid;
  constexpr int HPT = (2 * N3 + NT - 1) / NT;   // x-neighbour nodes per thread
  // Points of absent elements (and threads past the block's nodes) read the
  // block's first node, a valid state whose results are never stored.  The
  // loads are unconditional: a load under a condition is waited for where
  // the branches join.
  const int64_t lofs = act ? gofs : (int64_t)e0 * N3;
  double q[5], r[5], hq[HPT][5];
#pragma unroll
  for (int f = 0; f < 5; ++f) q[f] = Qin[f * EN3 + lofs];
#pragma unroll
  for (int h = 0; h < HPT; ++h) {
    const int x = tid + h * NT;
    if (x < 2 * N3) {
      const int right = x >= N3;
      const double* hb = Qin + (int64_t)(right ? exr : exl) * N3 + (x - right * N3);
#pragma unroll
      for (int f = 0; f < 5; ++f) hq[h][f] = hb[f * EN3];
    }
  }
  const int wave = tid >> 6, lane = tid & 63;
  constexpr bool PON = LINES == LINES_LDS && PairLines<N, EPB, NW>::on;
  // partner-lane pairs: on the point layout at even N, on the row-pair
  // layout at odd N (y/z slots only; one slot per face, one per wave)
  constexpr bool RP = LINES == LINES_DPP && N % 2 == 1;
  static_assert(!RP || (RowPairLane<N, EPB>::LANES <= 64 && S::NYZ == 4 && NW >= 4),
                "row pairs need one wave per y/z face");
  using PL = PairLines<N, EPB, NW>;
  double nb[PON ? 1 : RNDG][5];
  if constexpr (PON) {
    // y/z neighbour traces by point pairs, straight into the face-flux
    // region; phase B reads each back in the thread that then overwrites it
    // with the flux, so the region serves both without another barrier
    constexpr int F1 = PL::FS == 2 ? 3 : 5;
    switch (wave) {   // uniform over the wave
      case 0: pair_trace<N, EPB, 1, 0, F1>(Qin, EN3, eym, eyp, ne, lane, lmr, lpr, sH); break;
      case 1: pair_trace<N, EPB, 2, 0, F1>(Qin, EN3, ezm, ezp, ne, lane, lmr, lpr, sH); break;
      case 2: if (PL::FS == 2) pair_trace<N, EPB, 1, 3, 5>(Qin, EN3, eym, eyp, ne, lane, lmr, lpr, sH); break;
      case 3: if (PL::FS == 2) pair_trace<N, EPB, 2, 3, 5>(Qin, EN3, ezm, ezp, ne, lane, lmr, lpr, sH); break;
      default: break;
    }
  } else {
#pragma unroll
    for (int u = 0; u < RNDG; ++u) {
      const int s = wave + u * NW;
      const int i = (s < S::NYZ ? S::chunk(s) : 0) * 64 + lane;
      const int fel = i / N2, pt = i - fel * N2;
      const RowPairLane<N, EPB> rp(lane);
      if (RP && s < S::NYZ && rp.in && rp.fel < ne) {
        if constexpr (RP) {
          // (the two lanes of a pair share fel, and LANES is even)
          switch (S::face(s)) {   // uniform over the wave
            case 2: chunk_trace_rp<N, EPB, 1, 0>(Qin + (int64_t)eym * N3, EN3, rp, lmr, lpr, nb[u]); break;
            case 3: chunk_trace_rp<N, EPB, 1, 1>(Qin + (int64_t)eyp * N3, EN3, rp, lmr, lpr, nb[u]); break;
            case 4: chunk_trace_rp<N, EPB, 2, 0>(Qin + (int64_t)ezm * N3, EN3, rp, lmr, lpr, nb[u]); break;
            default: chunk_trace_rp<N, EPB, 2, 1>(Qin + (int64_t)ezp * N3, EN3, rp, lmr, lpr, nb[u]); break;
          }
        }
      } else if (!RP && s < S::NYZ && i < FP && fel < ne) {
        if constexpr (LINES == LINES_DPP && N % 2 == 0) {
          // (pairs of lanes share fel, and FP is even: both lanes of a pair
          // take this branch or neither)
          switch (S::face(s)) {   // uniform over the wave
            case 2: chunk_trace_x2<N, 1, 0>(Qin + (int64_t)eym * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
            case 3: chunk_trace_x2<N, 1, 1>(Qin + (int64_t)eyp * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
            case 4: chunk_trace_x2<N, 2, 0>(Qin + (int64_t)ezm * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
            default: chunk_trace_x2<N, 2, 1>(Qin + (int64_t)ezp * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
          }
        } else {
          switch (S::face(s)) {   // uniform over the wave
            case 2: chunk_trace<N, 1, 0>(Qin + (int64_t)eym * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
            case 3: chunk_trace<N, 1, 1>(Qin + (int64_t)eyp * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
            case 4: chunk_trace<N, 2, 0>(Qin + (int64_t)ezm * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
            default: chunk_trace<N, 2, 1>(Qin + (int64_t)ezp * N3, EN3, fel, pt, lmr, lpr, nb[u]); break;
          }
        }
      } else {
        nb[u][0] = 1.0; nb[u][1] = 0.0; nb[u][2] = 0.0; nb[u][3] = 0.0; nb[u][4] = 2.5;
      }
    }
  }
  // the 1-D tables, from uniform (scalar) kernarg reads: a per-thread
  // vector read would be waited for behind the neighbour loads above
  if (tid < N * N) {
    double v = 0.0;
#pragma unroll
    for (int x = 0; x < N * N; ++x) v = tid == x ? tb.Dh[x] : v;
    sDh[tid] = v;
  }
  if (tid < N) {
    double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      a = tid == m ? tb.lm[m] : a;
      b = tid == m ? tb.lp[m] : b;
      c = tid == m ? tb.liftm[m] : c;
      d = tid == m ? tb.liftp[m] : d;
    }
    sLm[tid] = a;
    sLp[tid] = b;
    sLiftm[tid] = c;
    sLiftp[tid] = d;
  }
  // stage the block (slots 1..ne) and its x-neighbours (slots 0 and ne + 1);
  // slots past ne + 1 stay unwritten: only points of absent elements read them
  if (act) {
#pragma unroll
    for (int f = 0; f < 5; ++f) sQ[f * NH + N3 + tid] = q[f];
  }
#pragma unroll
  for (int h = 0; h < HPT; ++h) {
    const int x = tid + h * NT;
    if (x < 2 * N3) {
      const int right = x >= N3;
      double* hs = sQ + (right ? ne + 1 : 0) * N3 + (x - right * N3);
#pragma unroll
      for (int f = 0; f < 5; ++f) hs[f * NH] = hq[h][f];
    }
  }
  __syncthreads();

  // ---- B: Lax-Friedrichs flux at every face point
#pragma unroll
  for (int u = 0; u < RND; ++u) {
    const int s = wave + u * NW;
    int i = (s < S::NS ? S::chunk(s) : 0) * 64 + lane;
    bool live = s < S::NS && i < FP;
    if constexpr (RP) {
      // y/z slots keep the row-pair layout of their neighbour traces
      if (s < S::NYZ) {
        const RowPairLane<N, EPB> rp(lane);
        live = rp.in && rp.c < N;
        i = rp.fel * N2 + rp.b * N + rp.c;
      }
    }
    if (live) {
      const int face = S::face(s);
      const int fel = i / N2, pt = i - fel * N2;
      const double* own = sQ + (fel + 1) * N3;
      double nbl[5];
      const double* nbv = nbl;
      if constexpr (PON) {
        if (face >= 2) {
#pragma unroll
          for (int f = 0; f < 5; ++f) nbl[f] = sH[(face * 5 + f) * FP + i];
        }
      } else {
        nbv = nb[u < RNDG ? u : 0];
      }
      const double g = tb.gamma, g1 = tb.gm1;
      double fs[5];
      switch (face) {   // uniform over the wave
        case 0: face_flux<N, 0, 0, true>(own, own - N3, nbv, NH, pt, sLm, sLp, g, g1, fs); break;
        case 1: face_flux<N, 0, 1, true>(own, own + N3, nbv, NH, pt, sLm, sLp, g, g1, fs); break;
        case 2: face_flux<N, 1, 0, false>(own, own, nbv, NH, pt, sLm, sLp, g, g1, fs); break;
        case 3: face_flux<N, 1, 1, false>(own, own, nbv, NH, pt, sLm, sLp, g, g1, fs); break;
        case 4: face_flux<N, 2, 0, false>(own, own, nbv, NH, pt, sLm, sLp, g, g1, fs); break;
        default: face_flux<N, 2, 1, false>(own, own, nbv, NH, pt, sLm, sLp, g, g1, fs); break;
      }
#pragma unroll
      for (int f = 0; f < 5; ++f) sH[(face * 5 + f) * FP + i] = fs[f];
    }
  }
  __syncthreads();   // last reads of sQ; sF reuses it

  // the residual, needed only in D: loaded here, its latency overlaps the
  // volume phase, and its registers are not held through the face phase
  // (unconditional in MODE 1: with `first` set it is read and ignored)
  if (MODE == 1) {
#pragma unroll
    for (int f = 0; f < 5; ++f) r[f] = RR[f * EN3 + lofs];
  } else {
#pragma unroll
    for (int f = 0; f < 5; ++f) r[f] = 0.0;
  }
  // ---- C: volume contraction + lift, one direction at a time
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
      for (int f = 0; f < 5; ++f) RR[f * EN3 + gofs] = acc[f];
    }
  } else {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      r[f] = (MODE == 2 || first) ? dt * acc[f] : fma(rka, r[f], dt * acc[f]);
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
