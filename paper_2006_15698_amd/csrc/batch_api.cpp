// Host side of the batched multi-mesh entry points (dg_batch_* in dg.h).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "dg_batch.h"

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct dg_batch {
  int count = 0;
  double gamma = 1.4;
  std::vector<DGBatchInst> inst;   // host copy (tables, offsets, dt)
  std::vector<int64_t> qoff;       // count + 1
  int epb_for_N[DG_MAXN + 1] = {0};
  std::vector<int2> items;
  hipStream_t stream = nullptr;
  int precision = DG_FP64;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool uploaded = false;
  // graphs: [parity] for one step each
  hipStream_t gstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  const double* gQ = nullptr;
  const double* gR = nullptr;
  int gprec = -1;
  unsigned grid[2] = {0, 0};   // persistent grid per precision (FP64, FP32 form)
  // launch form and visiting order of the work list (dg_batch_set_option).
  // Defaults: the fastest measured on the 512-mesh workload: one launch per
  // degree (20.1 against 14.5 GDOF-stages/s for the persistent launch in
  // FP64, 16.9 against 11.4 in the FP32 form), pencil order; the XCD remap
  // and the order move the per-degree rates by under 2%
  int xcd = 0;                 // each XCD walks its own contiguous part of the list
  int order = DG_ORDER_PENCIL; // item order within a mesh
  int pencil_x = 16;           // elements of a pencil along x (0 = whole row)
  int pencil_z = 8;            // element planes of a pencil along z
  int launch = DG_BATCH_PER_DEGREE;
  DGBatchSplit split{};
  int vbegin[DG_MAXN + 1] = {0}, vcount[DG_MAXN + 1] = {0};   // items per point count
};

namespace {

struct Layout {
  size_t off_inst, off_items, off_q2, total;
};

// Workspace: per-mesh records, the work list, and the second state buffer of
// the Q ping-pong (as long as the whole batch state).
Layout layout(const dg_batch* b) {
  Layout L;
  L.off_inst = 0;
  L.off_items = al256(sizeof(DGBatchInst) * b->count);
  L.off_q2 = L.off_items + al256(sizeof(int2) * b->items.size());
  L.total = L.off_q2 + al256((size_t)b->qoff[b->count] * sizeof(double));
  return L;
}

// The work list: meshes grouped by degree, highest first (workgroups that run
// at the same time mostly execute the same (N, tile) variant, and the
// costliest items come first); inside a mesh, blocks of up to epb
// consecutive elements of one x-row, visited row by row (DG_ORDER_LINEAR) or
// in pencils of pencil_x elements by pencil_z planes swept along y
// (DG_ORDER_PENCIL), so that an item's y- and z-neighbours are listed close
// to it.  Then, when the XCD split is on, the degree-mixed split below.
void build_items(dg_batch* b) {
  b->items.clear();
  std::vector<int> order(b->count);
  for (int i = 0; i < b->count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return b->inst[a].N > b->inst[c].N; });
  std::vector<int64_t> cost;
  for (int i : order) {
    DGBatchInst& I = b->inst[i];
    I.epb = b->epb_for_N[I.N];
    const int nx = I.tab.nx, ny = I.tab.ny, nz = I.tab.nz, epb = I.epb;
    const int nxb = (nx + epb - 1) / epb;
    const bool pencil = b->order == DG_ORDER_PENCIL;
    const int px = pencil && b->pencil_x > 0 && b->pencil_x < nx ? b->pencil_x : nx;
    const int tx = (px + epb - 1) / epb;
    const int tz = pencil ? std::min(std::max(b->pencil_z, 1), nz) : 1;
    const int64_t N3 = (int64_t)I.N * I.N * I.N;
    for (int pz = 0; pz < nz; pz += tz)
      for (int bx0 = 0; bx0 < nxb; bx0 += tx)
        for (int y = 0; y < ny; ++y)
          for (int z = pz; z < std::min(pz + tz, nz); ++z)
            for (int bx = bx0; bx < std::min(bx0 + tx, nxb); ++bx) {
              const int x0 = bx * epb;
              b->items.push_back(make_int2(i, (z * ny + y) * nx + x0));
              cost.push_back(std::min(epb, nx - x0) * N3);
            }
  }
  // XCD split: every degree group (contiguous in the list) is cut into 8
  // contiguous parts of equal node count, and XCD x gets part x of every
  // group, so each XCD runs the same mix of degrees (equal node counts of one
  // degree are equal work) on neighbouring items
  for (int N = 0; N <= DG_MAXN; ++N) b->vbegin[N] = b->vcount[N] = 0;
  for (size_t k = 0; k < b->items.size(); ++k) {
    const int N = b->inst[b->items[k].x].N;
    if (!b->vcount[N]) b->vbegin[N] = (int)k;
    ++b->vcount[N];
  }
  b->split.xcd = b->xcd && b->launch == DG_BATCH_PERSISTENT;
  if (b->split.xcd) {
    std::vector<int2> out;
    out.reserve(b->items.size());
    std::vector<size_t> group = {0};
    for (size_t k = 1; k < b->items.size(); ++k)
      if (b->inst[b->items[k].x].N != b->inst[b->items[k - 1].x].N) group.push_back(k);
    group.push_back(b->items.size());
    for (int x = 0; x < 8; ++x) {
      b->split.bounds[x] = (int)out.size();
      for (size_t gi = 0; gi + 1 < group.size(); ++gi) {
        int64_t total = 0;
        for (size_t k = group[gi]; k < group[gi + 1]; ++k) total += cost[k];
        const int64_t lo = total * x / 8, hi = total * (x + 1) / 8;
        int64_t acc = 0;   // node count before item k within the group
        for (size_t k = group[gi]; k < group[gi + 1]; ++k) {
          if (acc >= lo && acc < hi) out.push_back(b->items[k]);
          acc += cost[k];
        }
      }
    }
    b->split.bounds[8] = (int)out.size();
    b->items.swap(out);
  } else {
    for (int x = 0; x <= 8; ++x) b->split.bounds[x] = x == 8 ? (int)b->items.size() : 0;
  }
  b->uploaded = false;
}

void drop_graphs(dg_batch* b) {
  for (int k = 0; k < 2; ++k) {
    if (b->gexec[k]) (void)hipGraphExecDestroy(b->gexec[k]);
    b->gexec[k] = nullptr;
  }
  b->gQ = b->gR = nullptr;
}

DGBatchLaunch launch_of(const dg_batch* b, hipStream_t s) {
  const Layout L = layout(b);
  DGBatchLaunch l;
  l.inst = (const DGBatchInst*)(b->ws + L.off_inst);
  l.items = (const int2*)(b->ws + L.off_items);
  l.nitems = (int)b->items.size();
  l.f32 = b->precision == DG_FP32_MFMA;
  l.grid = b->grid[l.f32];
  l.stream = s;
  l.split = b->split;
  l.per_degree = b->launch == DG_BATCH_PER_DEGREE;
  l.xcd = b->xcd;
  for (int N = 0; N <= DG_MAXN; ++N) {
    l.vbegin[N] = b->vbegin[N];
    l.vcount[N] = b->vcount[N];
    l.epb[N] = b->epb_for_N[N];
  }
  // the XCD split needs the same number of workgroups on every XCD
  if (l.split.xcd) l.grid = l.grid >= 8 ? l.grid / 8 * 8 : 8;
  return l;
}

int ready(dg_batch* b) {
  if (!b) return dg_set_error(DG_EINVAL, "NULL batch");
  if (!b->ws) return dg_set_error(DG_EWORKSPACE, "no workspace set (need %zu bytes)", layout(b).total);
  if (!b->uploaded) return dg_set_error(DG_EWORKSPACE, "workspace not initialised (call dg_batch_set_workspace)");
  return DG_OK;
}

int hipfail(int err, const char* what) {
  return dg_set_error(DG_EHIP, "%s: HIP error %d (%s)", what, err, hipGetErrorString((hipError_t)err));
}

double* q2_of(const dg_batch* b) { return (double*)(b->ws + layout(b).off_q2); }

// The five stage launches of one step on stream s.  parity 0: the step
// starts from Q (and ends in Q2); parity 1: starts from Q2.
int launch_step(dg_batch* b, hipStream_t s, int parity, double* Q, double* res) {
  double* buf[2] = {Q, q2_of(b)};
  const DGBatchLaunch l = launch_of(b, s);
  for (int st = 0; st < 5; ++st) {
    const int g = parity + st;
    int err = dg_batch_launch_stage(l, 1, buf[g & 1], buf[(g + 1) & 1], res, kDgRKA[st], kDgRKB[st], st == 0);
    if (err) return err;
  }
  return 0;
}

}  // namespace

extern "C" {

dg_batch* dg_batch_create(int count, const int* n, const int* p, const double* L, double gamma) {
  if (count < 1 || !n || !p || !L) {
    dg_set_error(DG_EINVAL, "need count >= 1 and non-NULL n, p, L");
    return nullptr;
  }
  if (!(gamma > 1.0) || !std::isfinite(gamma)) {
    dg_set_error(DG_EINVAL, "gamma must be finite and > 1");
    return nullptr;
  }
  dg_batch* b = new (std::nothrow) dg_batch;
  if (!b) {
    dg_set_error(DG_EINVAL, "out of host memory");
    return nullptr;
  }
  b->count = count;
  b->gamma = gamma;
  b->inst.resize(count);
  b->qoff.resize(count + 1);
  for (int N = 1; N <= DG_MAXN; ++N) {
    int opts[16];
    const int k = dg_batch_tile_list(N, opts, 16);
    b->epb_for_N[N] = k ? opts[k - 1] : 0;   // default: the largest tile
  }
  int64_t q = 0;
  for (int i = 0; i < count; ++i) {
    const int nx = n[3 * i], ny = n[3 * i + 1], nz = n[3 * i + 2];
    const int64_t E = (int64_t)nx * ny * nz;
    if (nx < 1 || ny < 1 || nz < 1 || E > 0x7fffffffLL) {
      dg_set_error(DG_EINVAL, "mesh %d: bad size %d x %d x %d", i, nx, ny, nz);
      delete b;
      return nullptr;
    }
    if (p[i] < 1 || p[i] > 5) {
      dg_set_error(DG_EUNSUPPORTED, "mesh %d: batched degrees are 1..5 (got %d)", i, p[i]);
      delete b;
      return nullptr;
    }
    const double Li[3] = {L[3 * i], L[3 * i + 1], L[3 * i + 2]};
    if (!(Li[0] > 0) || !(Li[1] > 0) || !(Li[2] > 0)) {
      dg_set_error(DG_EINVAL, "mesh %d: domain lengths must be > 0", i);
      delete b;
      return nullptr;
    }
    DGBatchInst& I = b->inst[i];
    std::memset(&I, 0, sizeof(I));
    double xi[DG_MAXN], w[DG_MAXN];
    dg_build_tables(nx, ny, nz, p[i], gamma, Li, &I.tab, xi, w);
    I.N = p[i] + 1;
    const int64_t N3 = (int64_t)I.N * I.N * I.N;
    I.qoff = q;
    b->qoff[i] = q;
    q += 5 * E * N3;
    I.dt = 0.0;
  }
  b->qoff[count] = q;
  build_items(b);
  // The persistent grid holds the workgroups that can be resident at once
  // (compute units x workgroups per CU of that precision's kernel).
  int dev = 0, ncu = 0;
  const bool have_cu = hipGetDevice(&dev) == hipSuccess &&
                       hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0;
  for (int f32 = 0; f32 < 2; ++f32) b->grid[f32] = have_cu ? (unsigned)(ncu * dg_batch_blocks_per_cu(f32)) : 1024u;
  return b;
}

void dg_batch_destroy(dg_batch* b) {
  if (!b) return;
  drop_graphs(b);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->gstream) (void)hipStreamDestroy(b->gstream);
  delete b;
}

int dg_batch_set_stream(dg_batch* b, void* s) {
  if (!b) return dg_set_error(DG_EINVAL, "NULL batch");
  b->stream = (hipStream_t)s;
  return DG_OK;
}

int dg_batch_set_precision(dg_batch* b, int mode) {
  if (!b) return dg_set_error(DG_EINVAL, "NULL batch");
  if (mode != DG_FP64 && mode != DG_FP32_MFMA) return dg_set_error(DG_EINVAL, "unknown precision mode %d", mode);
  if (mode != b->precision) drop_graphs(b);
  b->precision = mode;
  return DG_OK;
}

int dg_batch_tile_options(int p, int* out, int max) {
  if (p < 0 || p >= DG_MAXN || !out || max < 0) return 0;
  return dg_batch_tile_list(p + 1, out, max);
}

int dg_batch_set_tile(dg_batch* b, int p, int epb) {
  if (!b) return dg_set_error(DG_EINVAL, "NULL batch");
  if (p < 1 || p > 5) return dg_set_error(DG_EINVAL, "degree must be 1..5");
  int opts[16];
  const int k = dg_batch_tile_list(p + 1, opts, 16);
  bool ok = false;
  for (int i = 0; i < k; ++i) ok = ok || opts[i] == epb;
  if (!ok) return dg_set_error(DG_EUNSUPPORTED, "tile %d not built for p=%d", epb, p);
  b->epb_for_N[p + 1] = epb;
  build_items(b);
  drop_graphs(b);
  b->ws = nullptr;   // the work list changed size: a workspace must be set again
  b->ws_bytes = 0;
  return DG_OK;
}

int dg_batch_set_option(dg_batch* b, int key, int value) {
  if (!b) return dg_set_error(DG_EINVAL, "NULL batch");
  switch (key) {
    case DG_OPT_XCD_REMAP: b->xcd = value ? 1 : 0; break;
    case DG_OPT_ORDER:
      if (value != DG_ORDER_LINEAR && value != DG_ORDER_PENCIL) return dg_set_error(DG_EINVAL, "unknown order %d", value);
      b->order = value;
      break;
    case DG_OPT_PENCIL_X:
      if (value < 0) return dg_set_error(DG_EINVAL, "pencil x extent %d < 0", value);
      b->pencil_x = value;
      break;
    case DG_OPT_PENCIL_Z:
      if (value < 1) return dg_set_error(DG_EINVAL, "pencil z extent %d < 1", value);
      b->pencil_z = value;
      break;
    case DG_OPT_BATCH_LAUNCH:
      if (value != DG_BATCH_PERSISTENT && value != DG_BATCH_PER_DEGREE)
        return dg_set_error(DG_EINVAL, "unknown batch launch form %d", value);
      b->launch = value;
      break;
    default: return dg_set_error(DG_EINVAL, "unknown batch option %d", key);
  }
  // the work list is rebuilt in place (same length): re-upload it
  build_items(b);
  drop_graphs(b);
  if (b->ws) {
    const Layout L = layout(b);
    int err = (int)hipStreamSynchronize(b->stream);
    if (err) return hipfail(err, "sync before work-list upload");
    err = (int)hipMemcpy(b->ws + L.off_items, b->items.data(), sizeof(int2) * b->items.size(), hipMemcpyHostToDevice);
    if (err) return hipfail(err, "upload work list");
    b->uploaded = true;
  }
  return DG_OK;
}

int dg_batch_get_option(const dg_batch* b, int key, int* value) {
  if (!b || !value) return dg_set_error(DG_EINVAL, "NULL argument");
  switch (key) {
    case DG_OPT_XCD_REMAP: *value = b->xcd; return DG_OK;
    case DG_OPT_BATCH_LAUNCH: *value = b->launch; return DG_OK;
    case DG_OPT_ORDER: *value = b->order; return DG_OK;
    case DG_OPT_PENCIL_X: *value = b->pencil_x; return DG_OK;
    case DG_OPT_PENCIL_Z: *value = b->pencil_z; return DG_OK;
    default: return dg_set_error(DG_EINVAL, "unknown batch option %d", key);
  }
}

int64_t dg_batch_offset(const dg_batch* b, int i) {
  if (!b || i < 0 || i > b->count) return -1;
  return b->qoff[i];
}

size_t dg_batch_workspace_bytes(const dg_batch* b) {
  if (!b) return 0;
  return layout(b).total;
}

int dg_batch_set_workspace(dg_batch* b, void* dptr, size_t bytes) {
  if (!b) return dg_set_error(DG_EINVAL, "NULL batch");
  if (!dptr) return dg_set_error(DG_EINVAL, "NULL workspace");
  if (((uintptr_t)dptr) & 255) return dg_set_error(DG_EINVAL, "workspace not 256-byte aligned");
  const Layout L = layout(b);
  if (bytes < L.total) return dg_set_error(DG_EWORKSPACE, "workspace %zu bytes < %zu", bytes, L.total);
  b->ws = (char*)dptr;
  b->ws_bytes = bytes;
  drop_graphs(b);
  int err = (int)hipMemcpy(b->ws + L.off_inst, b->inst.data(), sizeof(DGBatchInst) * b->count, hipMemcpyHostToDevice);
  if (err) return hipfail(err, "upload tables");
  err = (int)hipMemcpy(b->ws + L.off_items, b->items.data(), sizeof(int2) * b->items.size(), hipMemcpyHostToDevice);
  if (err) return hipfail(err, "upload work list");
  b->uploaded = true;
  return DG_OK;
}

int dg_batch_set_dt(dg_batch* b, const double* dt) {
  int rc = ready(b);
  if (rc) return rc;
  if (!dt) return dg_set_error(DG_EINVAL, "NULL dt");
  for (int i = 0; i < b->count; ++i) {
    if (!std::isfinite(dt[i])) return dg_set_error(DG_EINVAL, "dt[%d] not finite", i);
    b->inst[i].dt = dt[i];
  }
  const Layout L = layout(b);
  int err = (int)hipStreamSynchronize(b->stream);
  if (err) return hipfail(err, "sync before dt upload");
  err = (int)hipMemcpy(b->ws + L.off_inst, b->inst.data(), sizeof(DGBatchInst) * b->count, hipMemcpyHostToDevice);
  if (err) return hipfail(err, "upload dt");
  return DG_OK;
}

int dg_batch_rhs(dg_batch* b, const double* Q, double* R) {
  int rc = ready(b);
  if (rc) return rc;
  if (!Q || !R) return dg_set_error(DG_EINVAL, "NULL array");
  if (((uintptr_t)Q | (uintptr_t)R) & 7) return dg_set_error(DG_EINVAL, "arrays must be 8-byte aligned");
  const size_t sb = (size_t)b->qoff[b->count] * sizeof(double);
  if ((const char*)Q < (const char*)R + sb && (const char*)R < (const char*)Q + sb)
    return dg_set_error(DG_EALIAS, "R overlaps Q");
  const DGBatchLaunch l = launch_of(b, b->stream);
  int err = dg_batch_launch_stage(l, 0, Q, nullptr, R, 0.0, 0.0, 0);
  if (err) return hipfail(err, "batch rhs launch");
  return DG_OK;
}

int dg_batch_rk_steps(dg_batch* b, double* Q, double* res, int nsteps) {
  int rc = ready(b);
  if (rc) return rc;
  if (!Q || !res) return dg_set_error(DG_EINVAL, "NULL array");
  if (((uintptr_t)Q | (uintptr_t)res) & 7) return dg_set_error(DG_EINVAL, "arrays must be 8-byte aligned");
  if (nsteps < 0) return dg_set_error(DG_EINVAL, "nsteps must be >= 0");
  const size_t sb = (size_t)b->qoff[b->count] * sizeof(double);
  if ((char*)Q < (char*)res + sb && (char*)res < (char*)Q + sb) return dg_set_error(DG_EALIAS, "res overlaps Q");
  if (nsteps == 0) return DG_OK;
  int err = 0;
  for (int n = 0; n < nsteps; ++n) {
    err = launch_step(b, b->stream, n & 1, Q, res);
    if (err) return hipfail(err, "batch stage launch");
  }
  if (nsteps & 1) {
    err = (int)hipMemcpyAsync(Q, q2_of(b), sb, hipMemcpyDeviceToDevice, b->stream);
    if (err) return hipfail(err, "state copy");
  }
  return DG_OK;
}

int dg_batch_graph_steps(dg_batch* b, double* Q, double* res, int nsteps) {
  int rc = ready(b);
  if (rc) return rc;
  if (!Q || !res) return dg_set_error(DG_EINVAL, "NULL array");
  if (((uintptr_t)Q | (uintptr_t)res) & 7) return dg_set_error(DG_EINVAL, "arrays must be 8-byte aligned");
  if (nsteps < 0) return dg_set_error(DG_EINVAL, "nsteps must be >= 0");
  const size_t sb = (size_t)b->qoff[b->count] * sizeof(double);
  if ((char*)Q < (char*)res + sb && (char*)res < (char*)Q + sb) return dg_set_error(DG_EALIAS, "res overlaps Q");
  if (nsteps == 0) return DG_OK;
  int err;
  if (!b->gstream) {
    err = (int)hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking);
    if (err) return hipfail(err, "graph stream");
    err = (int)hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
    if (err) return hipfail(err, "graph event");
    err = (int)hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
    if (err) return hipfail(err, "graph event");
  }
  if (b->gQ != Q || b->gR != res || b->gprec != b->precision) drop_graphs(b);
  // order after the caller's stream
  err = (int)hipEventRecord(b->ev_in, b->stream);
  if (err) return hipfail(err, "event record");
  err = (int)hipStreamWaitEvent(b->gstream, b->ev_in, 0);
  if (err) return hipfail(err, "stream wait");
  for (int par = 0; par < 2; ++par) {
    if (b->gexec[par]) continue;
    hipGraph_t graph = nullptr;
    err = (int)hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal);
    if (err) return hipfail(err, "begin capture");
    int lerr = launch_step(b, b->gstream, par, Q, res);
    err = (int)hipStreamEndCapture(b->gstream, &graph);
    if (lerr) {
      if (graph) (void)hipGraphDestroy(graph);
      return hipfail(lerr, "capture launch");
    }
    if (err) return hipfail(err, "end capture");
    err = (int)hipGraphInstantiate(&b->gexec[par], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (err) return hipfail(err, "graph instantiate");
  }
  b->gQ = Q;
  b->gR = res;
  b->gprec = b->precision;
  for (int n = 0; n < nsteps; ++n) {
    err = (int)hipGraphLaunch(b->gexec[n & 1], b->gstream);
    if (err) return hipfail(err, "graph launch");
  }
  if (nsteps & 1) {
    err = (int)hipMemcpyAsync(Q, q2_of(b), sb, hipMemcpyDeviceToDevice, b->gstream);
    if (err) return hipfail(err, "state copy");
  }
  err = (int)hipEventRecord(b->ev_out, b->gstream);
  if (err) return hipfail(err, "event record");
  err = (int)hipStreamWaitEvent(b->stream, b->ev_out, 0);
  if (err) return hipfail(err, "stream wait");
  return DG_OK;
}

}  // extern "C"
