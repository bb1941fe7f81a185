// Host check of the paired neighbour-line lane maps (dgdev::PairLane and
// dgdev::PairLines, and the partner-lane pairs of chunk_trace_x2, compiled
// from the kernel's header).  LDS-handed pairs: for every degree
// and block size of the single-mesh and batched stage kernels, and both
// face directions that use it, the lanes of a wave cover every point of
// both faces of the block exactly once, each pair lies in one row, and the
// two points' line nodes are neighbours in memory inside the element for
// every m (so one 16-byte load fetches both).  Exit status 0 and "ok" on
// success.
#include <cstdio>
#include <vector>

#include "stage_nb.h"

template <int N, int EPB, int NT>
static int check() {
  using PL = dgdev::PairLines<N, EPB, NT / 64>;
  if (!PL::on) return 0;
  constexpr int N2 = N * N, N3 = N2 * N, FP = EPB * N2;
  if (2 * PL::LPF > 64) {
    printf("N=%d EPB=%d: pairs of two faces do not fit a wave\n", N, EPB);
    return 1;
  }
  for (int d = 1; d <= 2; ++d) {
    std::vector<int> hits(2 * FP, 0);
    for (int lane = 0; lane < 2 * PL::LPF; ++lane) {
      const dgdev::PairLane<N, EPB> p(lane);
      if (p.side < 0 || p.side > 1 || p.fel < 0 || p.fel >= EPB || p.pt < 0 || p.pt + 1 >= N2 ||
          p.pt % N + 1 >= N) {
        printf("N=%d EPB=%d lane %d: pair out of range\n", N, EPB, lane);
        return 1;
      }
      for (int m = 0; m < N; ++m) {
        const int n0 = d == 1 ? dgdev::tnode<N>(1, m, p.pt) : dgdev::tnode<N>(2, m, p.pt);
        const int n1 = d == 1 ? dgdev::tnode<N>(1, m, p.pt + 1) : dgdev::tnode<N>(2, m, p.pt + 1);
        if (n1 != n0 + 1 || n0 < 0 || n1 >= N3) {
          printf("N=%d EPB=%d d=%d lane %d m %d: line nodes %d, %d not adjacent\n", N, EPB, d, lane, m, n0, n1);
          return 1;
        }
      }
      const int base = p.side * FP + p.fel * N2 + p.pt;
      if (!p.dup) hits[base] += 1;
      hits[base + 1] += 1;
    }
    for (int i = 0; i < 2 * FP; ++i) {
      if (hits[i] != 1) {
        printf("N=%d EPB=%d d=%d: face point %d written %d times\n", N, EPB, d, i, hits[i]);
        return 1;
      }
    }
  }
  return 0;
}

// Partner-lane pairs (chunk_trace_x2, even N): the even point pe of every
// pair and pe + 1 lie in one row, and their line nodes are neighbours in
// memory at an even offset inside the element for every m (so the pair is
// 16-byte aligned whenever the element is, N^3 being even).
template <int N>
static int check_x2() {
  constexpr int N2 = N * N, N3 = N2 * N;
  static_assert(N3 % 2 == 0, "even element size");
  for (int d = 1; d <= 2; ++d) {
    for (int pe = 0; pe < N2; pe += 2) {
      if (pe % N + 1 >= N) {
        printf("N=%d: pair at %d leaves its row\n", N, pe);
        return 1;
      }
      for (int m = 0; m < N; ++m) {
        const int n0 = d == 1 ? dgdev::tnode<N>(1, m, pe) : dgdev::tnode<N>(2, m, pe);
        const int n1 = d == 1 ? dgdev::tnode<N>(1, m, pe + 1) : dgdev::tnode<N>(2, m, pe + 1);
        if (n1 != n0 + 1 || n0 % 2 != 0 || n1 >= N3) {
          printf("N=%d d=%d m=%d: pair at %d not an aligned pair of nodes (%d, %d)\n", N, d, m, pe, n0, n1);
          return 1;
        }
      }
    }
  }
  return 0;
}

// Row-pair layout (RowPairLane, odd N): lanes 2k and 2k + 1 share element
// and row and load the same node pair, starting at the even point of the
// pair's two lanes; the real lanes (c < N) cover every point of the face
// chunk exactly once, each owning half c & 1 of its pair; and for every line
// position m <= N - 2 (the ones loaded in pairs) the pair's line nodes are
// neighbours in memory inside the element (the last pair of a row reaches
// one node past the row).
template <int N, int EPB>
static int check_rp() {
  using RP = dgdev::RowPairLane<N, EPB>;
  constexpr int N2 = N * N, N3 = N2 * N;
  if (RP::LANES > 64 || RP::LANES % 2 != 0) {
    printf("N=%d EPB=%d: row-pair layout does not fit a wave\n", N, EPB);
    return 1;
  }
  std::vector<int> hits(EPB * N2, 0);
  for (int lane = 0; lane < RP::LANES; lane += 2) {
    const RP p0(lane), p1(lane + 1);
    if (!p0.in || !p1.in || p0.fel != p1.fel || p0.b != p1.b || p0.pair_start() != p1.pair_start()) {
      printf("N=%d EPB=%d lanes %d, %d: not one pair\n", N, EPB, lane, lane + 1);
      return 1;
    }
    const int ps = p0.pair_start();
    if (ps - N * p0.b < 0 || ps - N * p0.b > N - 1) {
      printf("N=%d EPB=%d lane %d: pair does not start in its row\n", N, EPB, lane);
      return 1;
    }
    for (int d = 1; d <= 2; ++d) {
      for (int m = 0; m + 1 < N; ++m) {
        const int n0 = d == 1 ? dgdev::tnode<N>(1, m, ps) : dgdev::tnode<N>(2, m, ps);
        const int n1 = n0 + 1;
        if (n0 < 0 || n1 >= N3) {
          printf("N=%d EPB=%d d=%d lane %d m %d: pair outside the element\n", N, EPB, d, lane, m);
          return 1;
        }
      }
    }
    for (const RP* p : {&p0, &p1}) {
      const int op = p->own_point();
      if (op - N * p->b < 0 || op - N * p->b > N - 1) {
        printf("N=%d EPB=%d: own point outside its row\n", N, EPB);
        return 1;
      }
      if (p->c < N) {
        if (ps + (p->c & 1) != p->c + N * p->b || op != p->c + N * p->b) {
          printf("N=%d EPB=%d: lane's own half is not its point\n", N, EPB);
          return 1;
        }
        hits[p->fel * N2 + p->c + N * p->b] += 1;
      }
    }
  }
  for (int i = 0; i < EPB * N2; ++i) {
    if (hits[i] != 1) {
      printf("N=%d EPB=%d: point %d covered %d times\n", N, EPB, i, hits[i]);
      return 1;
    }
  }
  return 0;
}

int main() {
  int bad = 0;
  bad |= check_rp<5, 2>() | check_rp<5, 1>() | check_rp<7, 1>() | check_rp<3, 4>();
  bad |= check_x2<2>() | check_x2<4>() | check_x2<6>() | check_x2<8>();
  // single-mesh kernels (degree, elements per block, threads)
  bad |= check<2, 16, 128>() | check<3, 9, 256>() | check<4, 4, 256>() | check<5, 2, 256>();
  bad |= check<6, 1, 256>() | check<7, 1, 384>() | check<8, 1, 512>();
  // batched kernel variants (256 threads)
  bad |= check<2, 8, 256>() | check<2, 16, 256>() | check<3, 4, 256>() | check<3, 9, 256>();
  bad |= check<4, 2, 256>() | check<4, 4, 256>() | check<5, 1, 256>() | check<5, 2, 256>() | check<6, 1, 256>();
  if (bad) return 1;
  printf("ok\n");
  return 0;
}
