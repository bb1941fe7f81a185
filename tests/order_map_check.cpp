// Host check of the stage kernel's element-block visiting order
// (dgdev::block_elements, compiled from the kernel's header): for every
// mesh, pencil shape, block size and XCD setting below, each element is
// covered by exactly one workgroup, blocks are non-empty, in range and lie
// in one x-row, and the index order without XCD chunks visits blocks by
// increasing first element.  Exit status 0 and "ok" on success.
#include <cstdio>
#include <vector>

#include "stage_nb.h"

template <int EPB>
static int check(int nx, int ny, int nz, int pencil_x, int pencil_z, int xcd) {
  dg_ctx c{};
  c.nx = nx; c.ny = ny; c.nz = nz;
  c.E = (int64_t)nx * ny * nz;
  c.pencil_x = pencil_x; c.pencil_z = pencil_z; c.xcd_remap = xcd;
  DGTables tb{};
  tb.nx = nx; tb.ny = ny; tb.nz = nz; tb.E = (int)c.E;
  for (int order = 0; order < 2; ++order) {
    c.order = order;
    unsigned grid;
    const DGOrder o = dg_order(&c, EPB, &grid);
    std::vector<int> hits(c.E, 0);
    int last = -1;
    for (unsigned w = 0; w < grid; ++w) {
      int e0, ne;
      dgdev::block_elements<EPB>(tb, o, (int)w, (int)grid, e0, ne);
      if (ne < 1 || ne > EPB || e0 < 0 || e0 + ne > c.E) {
        printf("block %u out of range: e0 %d ne %d\n", w, e0, ne);
        return 1;
      }
      if (e0 / nx != (e0 + ne - 1) / nx) {
        printf("block %u leaves its row\n", w);
        return 1;
      }
      if (order == DG_ORDER_LINEAR && !xcd && e0 <= last) {
        printf("index order not increasing at block %u\n", w);
        return 1;
      }
      last = e0;
      for (int k = 0; k < ne; ++k) hits[e0 + k]++;
    }
    for (int64_t e = 0; e < c.E; ++e)
      if (hits[e] != 1) {
        printf("element %lld visited %d times (mesh %dx%dx%d pencil %dx%d xcd %d order %d EPB %d)\n",
               (long long)e, hits[e], nx, ny, nz, pencil_x, pencil_z, xcd, order, EPB);
        return 1;
      }
  }
  return 0;
}

int main() {
  const int dims[] = {1, 2, 3, 5, 8, 13, 24};
  int cases = 0;
  for (int nx : dims)
    for (int ny : dims)
      for (int nz : dims)
        for (int px : {0, 1, 3, 17})
          for (int pz : {1, 2, 6, 40})
            for (int xcd : {0, 1}) {
              if (check<1>(nx, ny, nz, px, pz, xcd) || check<2>(nx, ny, nz, px, pz, xcd) ||
                  check<4>(nx, ny, nz, px, pz, xcd) || check<9>(nx, ny, nz, px, pz, xcd) ||
                  check<16>(nx, ny, nz, px, pz, xcd))
                return 1;
              cases += 5;
            }
  if (check<2>(48, 48, 48, 0, 6, 1) || check<4>(32, 32, 32, 16, 8, 1) || check<1>(40, 40, 40, 8, 5, 0)) return 1;
  printf("%d cases ok\n", cases + 3);
  return 0;
}
