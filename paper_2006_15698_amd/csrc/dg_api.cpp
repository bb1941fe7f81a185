// Host side of the C ABI declared in include/dg.h: argument validation,
// constant tables, workspace carve-up and kernel sequencing.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "dg_batch.h"
#include "dg_internal.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(int err, const char* what) {
  return fail(DG_EHIP, "%s: HIP error %d (%s)", what, err, hipGetErrorString((hipError_t)err));
}

// Per-launch HIP-event timing (dg_set_timing).
enum { TK_TRACE = 0, TK_STAGE = 1, TK_RHS = 2, TK_VJP = 3, TK_RED = 4, TK_STAGE_FIRST = 5, TK_VISC = 6, TK_NKIND = 7 };
constexpr size_t kMaxTimed = 65536;

struct DGTiming {
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  std::vector<int> kind;
  size_t used = 0;
  ~DGTiming() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

// Run `launch` (returning a hipError_t as int), bracketed by events when
// timing is on.
template <class F>
int timed(dg_ctx* c, int kind, F&& launch) {
  if (!c->timing_on) return launch();
  DGTiming* T = (DGTiming*)c->timing;
  if (T->used >= kMaxTimed) return launch();
  if (T->ev.size() < 2 * (T->used + 1)) {
    hipEvent_t a, b;
    int err = (int)hipEventCreate(&a);
    if (err) return err;
    err = (int)hipEventCreate(&b);
    if (err) return err;
    T->ev.push_back(a);
    T->ev.push_back(b);
  }
  hipEvent_t a = T->ev[2 * T->used], b = T->ev[2 * T->used + 1];
  int err = (int)hipEventRecord(a, c->stream);
  if (err) return err;
  err = launch();
  if (err) return err;
  err = (int)hipEventRecord(b, c->stream);
  if (err) return err;
  if (T->kind.size() <= T->used) T->kind.push_back(kind);
  else T->kind[T->used] = kind;
  T->used++;
  return 0;
}

// Carpenter-Kennedy (5,4) 2N-storage coefficients: the five-stage fourth-order
// low-storage scheme named in Sections IV-V (coefficients not printed in the
// paper; the standard published values).
const double kRKA[5] = {0.0,
                        -567301805773.0 / 1357537059087.0,
                        -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0,
                        -1275806237668.0 / 842570457699.0};
const double kRKB[5] = {1432997174477.0 / 9575080441755.0,
                        5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0,
                        3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};

// Legendre P_n(x) and P_n'(x) by the three-term recurrence.
void legendre(int n, double x, double* pn, double* dpn) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    *pn = 1.0;
    *dpn = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;
  *dpn = n * (x * p1 - p0) / (x * x - 1.0);
}

// N-point Gauss-Legendre rule (Section II-B): Newton iteration on P_N from
// Chebyshev-like initial guesses, weights 2 / ((1 - x^2) P_N'(x)^2).
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double pn, dpn;
      legendre(n, z, &pn, &dpn);
      const double dz = pn / dpn;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    double pn, dpn;
    legendre(n, z, &pn, &dpn);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dpn * dpn);
  }
  if (n % 2 == 1) x[n / 2] = 0.0;  // exact centre node for odd n
  // enforce the symmetry of the rule
  for (int i = 0; i < n / 2; ++i) {
    const double xs = 0.5 * (x[n - 1 - i] - x[i]);
    const double ws = 0.5 * (w[n - 1 - i] + w[i]);
    x[i] = -xs;
    x[n - 1 - i] = xs;
    w[i] = ws;
    w[n - 1 - i] = ws;
  }
}

void build_tables(dg_ctx* c) {
  dg_build_tables(c->nx, c->ny, c->nz, c->p, c->gamma, c->L, &c->tab, c->xi, c->w);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool overlap(const void* a, const void* b, size_t bytes) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + bytes && pb < pa + bytes;
}

// State arrays are arrays of doubles: the kernels read them in 8- and
// 16-byte pieces at 8-byte alignment.
bool misaligned(const void* p) { return ((uintptr_t)p & 7) != 0; }

int check_ready(dg_ctx* c) {
  if (!c) return fail(DG_EINVAL, "NULL context");
  const DGWorkspace L = dg_workspace_layout(c);
  if (!c->ws) return fail(DG_EWORKSPACE, "no workspace set (need %zu bytes)", L.total);
  if (c->ws_bytes < L.total) return fail(DG_EWORKSPACE, "workspace %zu bytes < %zu", c->ws_bytes, L.total);
  return DG_OK;
}

size_t state_bytes(const dg_ctx* c) { return (size_t)c->E * c->N * c->N * c->N * DG_NF * sizeof(double); }

double* trace_buf(dg_ctx* c, int which) {
  const DGWorkspace L = dg_workspace_layout(c);
  return (double*)(c->ws + (which ? L.off_trace1 : L.off_trace0));
}

int run_reduce(dg_ctx* c, const double* Q, double out[DG_RED_VALS]) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!Q) return fail(DG_EINVAL, "NULL state");
  if (misaligned(Q)) return fail(DG_EINVAL, "state is not 8-byte aligned");
  const DGWorkspace L = dg_workspace_layout(c);
  double* red = (double*)(c->ws + L.off_red);
  int err = timed(c, TK_RED, [&] { return dg_launch_reduce(c, Q, red); });
  if (err) return hip_fail(err, "reduce launch");
  err = (int)hipMemcpyAsync(out, red + DG_RED_BLOCKS * DG_RED_VALS, DG_RED_VALS * sizeof(double),
                            hipMemcpyDeviceToHost, c->stream);
  if (err) return hip_fail(err, "reduce copy");
  err = (int)hipStreamSynchronize(c->stream);
  if (err) return hip_fail(err, "reduce sync");
  return DG_OK;
}

double* q2_buf(dg_ctx* c) { return (double*)(c->ws + dg_workspace_layout(c).off_q2); }

// Neighbour-read sequencing: stage g reads buf[g % 2] and writes
// buf[(g + 1) % 2] with buf = {Q, Q2}; an odd count ends in Q2, copied back.
// Q2 is the workspace's second state buffer unless the caller names another
// one; with `timing` false no launch is bracketed by timing events (which are
// created on first use).
int stages_nb(dg_ctx* c, double* Q, double* res, double dt, int s0, int count, double* q2 = nullptr,
              bool timing = true) {
  double* buf[2] = {Q, q2 ? q2 : q2_buf(c)};
  int err = 0;
  for (int g = 0; g < count; ++g) {
    const int s = (s0 + g) % 5;
    auto launch = [&] {
      return c->precision == DG_FP32_MFMA
                 ? dg_launch_stage_nb_f32(c, buf[g & 1], buf[(g + 1) & 1], res, 1, kRKA[s], kRKB[s], dt, s == 0)
                 : dg_launch_stage_nb(c, buf[g & 1], buf[(g + 1) & 1], res, 1, kRKA[s], kRKB[s], dt, s == 0);
    };
    err = timing ? timed(c, s == 0 ? TK_STAGE_FIRST : TK_STAGE, launch) : launch();
    if (err) return hip_fail(err, "stage launch");
  }
  if (count & 1) {
    err = (int)hipMemcpyAsync(Q, buf[1], state_bytes(c), hipMemcpyDeviceToDevice, c->stream);
    if (err) return hip_fail(err, "state copy");
  }
  return DG_OK;
}

// Inviscid rate R = dQ/dt of the Euler terms: the split-form kernel, or the
// neighbour-read kernel (bitwise the same as the trace-buffer form).
int euler_rate_nb(dg_ctx* c, const double* Q, double* R) {
  if (c->volume_form == DG_VOLUME_KEP) return dg_launch_split(c, Q, nullptr, R, 0, 0.0, 0.0, 0.0);
  return c->precision == DG_FP32_MFMA ? dg_launch_stage_nb_f32(c, Q, nullptr, R, 0, 0.0, 0.0, 0.0, 0)
                                      : dg_launch_stage_nb(c, Q, nullptr, R, 0, 0.0, 0.0, 0.0, 0);
}

// Split-form stages: Q ping-pongs between Q and the workspace's second
// state buffer like the neighbour-read stages (an odd count ends with a
// copy back).
int stages_split(dg_ctx* c, double* Q, double* res, double dt, int s0, int count) {
  double* buf[2] = {Q, q2_buf(c)};
  for (int g = 0; g < count; ++g) {
    const int s = (s0 + g) % 5;
    int err = timed(c, s == 0 ? TK_STAGE_FIRST : TK_STAGE, [&] {
      return dg_launch_split(c, buf[g & 1], buf[(g + 1) & 1], res, s == 0 ? 2 : 1, kRKA[s], kRKB[s], dt);
    });
    if (err) return hip_fail(err, "split-form stage launch");
  }
  if (count & 1) {
    int err = (int)hipMemcpyAsync(Q, buf[1], state_bytes(c), hipMemcpyDeviceToDevice, c->stream);
    if (err) return hip_fail(err, "state copy");
  }
  return DG_OK;
}

// Whether the viscous-flux launch forms the inviscid rate too: the FP64
// standard form (the split form and the FP32 form have kernels of their own).
bool visc_fused(const dg_ctx* c) {
  return c->visc_fused && c->volume_form == DG_VOLUME_STANDARD && c->precision == DG_FP64;
}

// Navier-Stokes stages: per stage the inviscid rate into the workspace (in
// the viscous-flux launch, or before it), the viscous flux, and the viscous
// rate, combined with the inviscid one into the LSERK45 update of Q and res
// in place.
int stages_visc(dg_ctx* c, double* Q, double* res, double dt, int s0, int count) {
  const DGWorkspace L = dg_workspace_layout(c);
  double* R = (double*)(c->ws + L.off_visc_r);
  double* Fv = (double*)(c->ws + L.off_visc_fv);
  const bool fused = visc_fused(c);
  for (int g = 0; g < count; ++g) {
    const int s = (s0 + g) % 5;
    int err = 0;
    if (!fused) {
      err = timed(c, TK_RHS, [&] { return euler_rate_nb(c, Q, R); });
      if (err) return hip_fail(err, "inviscid rate launch");
    }
    err = timed(c, TK_VISC,
                [&] { return dg_launch_visc(c, Q, Fv, R, Q, res, 1, kRKA[s], kRKB[s], dt, s == 0, fused); });
    if (err) return hip_fail(err, "viscous stage launch");
  }
  return DG_OK;
}

int stages(dg_ctx* c, double* Q, double* res, double dt, int s0, int count) {
  // Traces of the initial Q, then `count` stages starting at stage s0; each
  // stage but the last writes the traces of its updated Q for the next.
  const bool f32 = c->precision == DG_FP32_MFMA;
  if (c->mu > 0.0) return stages_visc(c, Q, res, dt, s0, count);
  if (c->volume_form == DG_VOLUME_KEP) return stages_split(c, Q, res, dt, s0, count);
  if (c->exchange == DG_EXCHANGE_NEIGHBOUR) return stages_nb(c, Q, res, dt, s0, count);
  int err = timed(c, TK_TRACE, [&] {
    return f32 ? dg_launch_trace_f32(c, Q, (char*)trace_buf(c, 0)) : dg_launch_trace(c, Q, trace_buf(c, 0));
  });
  if (err) return hip_fail(err, "trace launch");
  for (int g = 0; g < count; ++g) {
    const int s = (s0 + g) % 5;
    double* tin = trace_buf(c, g & 1);
    double* tout = g + 1 < count ? trace_buf(c, (g + 1) & 1) : nullptr;
    err = timed(c, s == 0 ? TK_STAGE_FIRST : TK_STAGE, [&] {
      return f32 ? dg_launch_stage_f32(c, Q, res, (const char*)tin, (char*)tout, kRKA[s], kRKB[s], dt, s == 0)
                 : dg_launch_stage(c, Q, res, tin, tout, kRKA[s], kRKB[s], dt, s == 0);
    });
    if (err) return hip_fail(err, "stage launch");
  }
  return DG_OK;
}

// Second state buffer for dg_rk_steps_noalloc: a file-scope device array,
// one copy on every GPU the library runs on, kept until the process ends.  In
// host code `scratch` names a host-side stand-in, not the device memory: the
// device address is looked up once per device with hipGetSymbolAddress (while
// that device is current) and only that address is ever handed to kernels
// and copies.
constexpr size_t kScratchBytes = DG_NOALLOC_MAX_BYTES;
__device__ __align__(256) static double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

int scratch_of_current_device(double** out) {
  int dev = 0;
  int err = (int)hipGetDevice(&dev);
  if (err) return hip_fail(err, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(DG_EUNSUPPORTED, "device ordinal %d >= %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    err = (int)hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err) return hip_fail(err, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(DG_EHIP, "hipGetSymbolAddress(scratch) gave NULL");
    g_scratch_dev[dev] = (double*)p;
  }
  *out = g_scratch_dev[dev];
  return DG_OK;
}

int check_state_pair(dg_ctx* c, const void* a, const char* an, const void* b, const char* bn) {
  if (!a || !b) return fail(DG_EINVAL, "NULL %s", !a ? an : bn);
  if (misaligned(a) || misaligned(b)) return fail(DG_EINVAL, "%s is not 8-byte aligned", misaligned(a) ? an : bn);
  if (overlap(a, b, state_bytes(c))) return fail(DG_EALIAS, "%s overlaps %s", an, bn);
  return DG_OK;
}

}  // namespace

void dg_build_tables(int nx, int ny, int nz, int p, double gamma, const double L[3], DGTables* tp, double* xi,
                     double* w) {
  const int N = p + 1;
  DGTables& t = *tp;
  std::memset(&t, 0, sizeof(t));
  gauss_legendre(N, xi, w);
  // barycentric weights 1 / prod_{m != i} (xi_i - xi_m)
  double bw[DG_MAXN];
  for (int i = 0; i < N; ++i) {
    double prod = 1.0;
    for (int m = 0; m < N; ++m)
      if (m != i) prod *= (xi[i] - xi[m]);
    bw[i] = 1.0 / prod;
  }
  // D[a][i] = l_i'(xi_a): off-diagonal (bw_i / bw_a) / (xi_a - xi_i),
  // diagonal from the zero row sum (derivative of a constant).
  double D[DG_MAXN][DG_MAXN];
  for (int a = 0; a < N; ++a) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) {
      if (i == a) continue;
      D[a][i] = (bw[i] / bw[a]) / (xi[a] - xi[i]);
      s += D[a][i];
    }
    D[a][a] = -s;
  }
  for (int i = 0; i < N; ++i) {
    double lm = 1.0, lp = 1.0;
    for (int m = 0; m < N; ++m) {
      if (m == i) continue;
      lm *= (-1.0 - xi[m]) / (xi[i] - xi[m]);
      lp *= (1.0 - xi[m]) / (xi[i] - xi[m]);
    }
    t.lm[i] = lm;
    t.lp[i] = lp;
    t.liftm[i] = lm / w[i];
    t.liftp[i] = lp / w[i];
    t.w[i] = w[i];
    for (int a = 0; a < N; ++a) t.Dh[i * N + a] = w[a] * D[a][i] / w[i];
  }
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int a = 0; a < N; ++a) {
      s += t.Dh[i * N + a];
      t.Dh32[i * N + a] = (float)t.Dh[i * N + a];
    }
    t.rs[i] = s;
    t.lm32[i] = (float)t.lm[i];
    t.lp32[i] = (float)t.lp[i];
  }
  const double h[3] = {L[0] / nx, L[1] / ny, L[2] / nz};
  for (int d = 0; d < 3; ++d) {
    t.sc[d] = 2.0 / h[d];
    t.hinv[d] = 1.0 / h[d];
  }
  t.J = h[0] * h[1] * h[2] / 8.0;
  t.gamma = gamma;
  t.gm1 = gamma - 1.0;
  t.nx = nx;
  t.ny = ny;
  t.nz = nz;
  t.E = nx * ny * nz;
}

const double kDgRKA[5] = {kRKA[0], kRKA[1], kRKA[2], kRKA[3], kRKA[4]};
const double kDgRKB[5] = {kRKB[0], kRKB[1], kRKB[2], kRKB[3], kRKB[4]};

int dg_set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

DGWorkspace dg_workspace_layout(const dg_ctx* c) {
  DGWorkspace L;
  const size_t N2 = (size_t)c->N * c->N;
  const size_t N3 = N2 * c->N;
  L.trace_bytes = align256(30 * N2 * (size_t)c->E * sizeof(double));
  L.off_trace0 = 0;
  L.off_trace1 = L.off_trace0 + L.trace_bytes;
  L.off_red = L.off_trace1 + L.trace_bytes;
  const size_t red_bytes = align256((DG_RED_BLOCKS + 1) * DG_RED_VALS * sizeof(double));
  L.off_vjp = L.off_red + red_bytes;
  // adjoint scratch for the reverse RK stage: two state-sized buffers
  const size_t vjp_bytes = 2 * align256(DG_NF * N3 * (size_t)c->E * sizeof(double));
  L.off_q2 = L.off_vjp + vjp_bytes;
  L.total = L.off_q2 + align256(DG_NF * N3 * (size_t)c->E * sizeof(double));
  L.off_visc_r = L.off_visc_fv = L.total;
  if (c->mu > 0.0) {
    L.off_visc_fv = L.off_visc_r + align256(DG_NF * N3 * (size_t)c->E * sizeof(double));
    L.total = L.off_visc_fv + align256(12 * N3 * (size_t)c->E * sizeof(double));
  }
  return L;
}

// r = 1/x and s = sqrt(x) elementwise with the flux kernels' recip/root
// (kern_check.hip).
int dg_launch_recip_root(hipStream_t stream, const double* x, double* r, double* s, int64_t n);

extern "C" {

const char* dg_last_error(void) { return g_err; }

dg_ctx* dg_create(int nx, int ny, int nz, int p, double gamma) {
  if (nx < 1 || ny < 1 || nz < 1) {
    fail(DG_EINVAL, "mesh sizes must be >= 1 (got %d x %d x %d)", nx, ny, nz);
    return nullptr;
  }
  if (p < 0 || p >= DG_MAXN) {
    fail(DG_EUNSUPPORTED, "p must be in 0..%d (got %d)", DG_MAXN - 1, p);
    return nullptr;
  }
  if (!(gamma > 1.0) || !std::isfinite(gamma)) {
    fail(DG_EINVAL, "gamma must be finite and > 1 (got %g)", gamma);
    return nullptr;
  }
  const int64_t E = (int64_t)nx * ny * nz;
  if (E > 0x7fffffffLL) {
    fail(DG_EUNSUPPORTED, "element count %lld exceeds 2^31-1", (long long)E);
    return nullptr;
  }
  dg_ctx* c = new (std::nothrow) dg_ctx;
  if (!c) {
    fail(DG_EINVAL, "out of host memory");
    return nullptr;
  }
  std::memset(c, 0, sizeof(*c));
  c->nx = nx;
  c->ny = ny;
  c->nz = nz;
  c->p = p;
  c->N = p + 1;
  c->E = E;
  c->gamma = gamma;
  c->L[0] = c->L[1] = c->L[2] = 1.0;
  c->stream = nullptr;
  c->precision = DG_FP64;
  c->exchange = DG_EXCHANGE_NEIGHBOUR;
  // Fastest measured on MI355X (32^3 p=3, 48^3 p=4, 40^3 p=6): pencils of
  // 16 x 8 elements, each XCD taking a contiguous part of the order.
  c->order = DG_ORDER_PENCIL;
  c->xcd_remap = 1;
  c->pencil_x = 16;
  c->pencil_z = 8;
  c->visc_fused = 1;
  c->mu = 0.0;
  c->prandtl = 0.72;
  c->kappa = 0.0;
  c->volume_form = DG_VOLUME_STANDARD;
  c->epoch = 1;
  c->gstream = nullptr;
  c->ev_in = c->ev_out = nullptr;
  c->gexec[0] = c->gexec[1] = nullptr;
  c->gQ = c->gR = nullptr;
  c->gdt = 0.0;
  c->gepoch = 0;
  build_tables(c);
  g_err[0] = 0;
  return c;
}

void dg_destroy(dg_ctx* c) {
  if (!c) return;
  delete (DGTiming*)c->timing;
  for (int k = 0; k < 2; ++k)
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  delete c;
}

int dg_set_timing(dg_ctx* c, int on) {
  if (!c) return fail(DG_EINVAL, "NULL context");
  if (on) {
    if (!c->timing) c->timing = new (std::nothrow) DGTiming;
    if (!c->timing) return fail(DG_EINVAL, "out of host memory");
    ((DGTiming*)c->timing)->used = 0;
  }
  c->timing_on = on ? 1 : 0;
  return DG_OK;
}

int dg_timing_read(dg_ctx* c, double ms[7], int64_t count[7]) {
  if (!c) return fail(DG_EINVAL, "NULL context");
  if (!ms || !count) return fail(DG_EINVAL, "NULL output");
  for (int k = 0; k < TK_NKIND; ++k) {
    ms[k] = 0.0;
    count[k] = 0;
  }
  DGTiming* T = (DGTiming*)c->timing;
  if (!T || T->used == 0) return DG_OK;
  int err = (int)hipEventSynchronize(T->ev[2 * T->used - 1]);
  if (err) return hip_fail(err, "timing sync");
  for (size_t u = 0; u < T->used; ++u) {
    float t = 0.f;
    err = (int)hipEventElapsedTime(&t, T->ev[2 * u], T->ev[2 * u + 1]);
    if (err) return hip_fail(err, "timing read");
    ms[T->kind[u]] += t;
    count[T->kind[u]] += 1;
  }
  return DG_OK;
}

int dg_set_domain(dg_ctx* c, double Lx, double Ly, double Lz) {
  if (!c) return fail(DG_EINVAL, "NULL context");
  if (!(Lx > 0) || !(Ly > 0) || !(Lz > 0) || !std::isfinite(Lx) || !std::isfinite(Ly) || !std::isfinite(Lz))
    return fail(DG_EINVAL, "domain lengths must be finite and > 0");
  c->L[0] = Lx;
  c->L[1] = Ly;
  c->L[2] = Lz;
  build_tables(c);
  ++c->epoch;
  return DG_OK;
}

int dg_set_stream(dg_ctx* c, void* s) {
  if (!c) return fail(DG_EINVAL, "NULL context");
  c->stream = (hipStream_t)s;
  return DG_OK;
}

int dg_set_precision(dg_ctx* c, int mode) {
  if (!c) return fail(DG_EINVAL, "NULL context");
  if (mode == DG_FP64) {
    c->precision = mode;
    ++c->epoch;
    return DG_OK;
  }
  if (mode == DG_FP32_MFMA) {
    if (!dg_f32_supported(c->N)) return fail(DG_EUNSUPPORTED, "FP32 matrix-core form not built for p=%d", c->p);
    if (c->volume_form == DG_VOLUME_KEP)
      return fail(DG_EUNSUPPORTED, "the split form runs in FP64 only (set DG_VOLUME_STANDARD first)");
    c->precision = mode;
    ++c->epoch;
    return DG_OK;
  }
  return fail(DG_EINVAL, "unknown precision mode %d", mode);
}

int dg_set_viscosity(dg_ctx* c, double mu, double prandtl) {
  if (!c) return fail(DG_EINVAL, "NULL context");
  if (!(mu >= 0.0) || !std::isfinite(mu)) return fail(DG_EINVAL, "viscosity must be finite and >= 0 (got %g)", mu);
  if (!(prandtl > 0.0) || !std::isfinite(prandtl))
    return fail(DG_EINVAL, "Prandtl number must be finite and > 0 (got %g)", prandtl);
  c->mu = mu;
  c->prandtl = prandtl;
  c->kappa = mu * (c->gamma / (c->gamma - 1.0)) / prandtl;
  ++c->epoch;
  return DG_OK;
}

int dg_set_volume_form(dg_ctx* c, int form) {
  if (!c) return fail(DG_EINVAL, "NULL context");
  if (form != DG_VOLUME_STANDARD && form != DG_VOLUME_KEP) return fail(DG_EINVAL, "unknown volume form %d", form);
  if (form == DG_VOLUME_KEP && c->precision == DG_FP32_MFMA)
    return fail(DG_EUNSUPPORTED, "the split form runs in FP64 only (precision is the FP32 form)");
  c->volume_form = form;
  ++c->epoch;
  return DG_OK;
}

int dg_set_option(dg_ctx* c, int key, int value) {
  if (!c) return fail(DG_EINVAL, "NULL context");
  if (key == DG_OPT_EXCHANGE) {
    if (value != DG_EXCHANGE_TRACES && value != DG_EXCHANGE_NEIGHBOUR)
      return fail(DG_EINVAL, "unknown exchange %d", value);
    c->exchange = value;
    ++c->epoch;
    return DG_OK;
  }
  if (key == DG_OPT_XCD_REMAP) {
    c->xcd_remap = value ? 1 : 0;
    ++c->epoch;
    return DG_OK;
  }
  if (key == DG_OPT_ORDER) {
    if (value != DG_ORDER_LINEAR && value != DG_ORDER_PENCIL) return fail(DG_EINVAL, "unknown order %d", value);
    c->order = value;
    ++c->epoch;
    return DG_OK;
  }
  if (key == DG_OPT_PENCIL_X) {
    if (value < 0) return fail(DG_EINVAL, "pencil x extent %d < 0", value);
    c->pencil_x = value;
    ++c->epoch;
    return DG_OK;
  }
  if (key == DG_OPT_PENCIL_Z) {
    if (value < 1) return fail(DG_EINVAL, "pencil z extent %d < 1", value);
    c->pencil_z = value;
    ++c->epoch;
    return DG_OK;
  }
  if (key == DG_OPT_VISC_FUSED) {
    c->visc_fused = value ? 1 : 0;
    ++c->epoch;
    return DG_OK;
  }
  return fail(DG_EINVAL, "unknown option %d", key);
}

int dg_get_option(const dg_ctx* c, int key, int* value) {
  if (!c || !value) return fail(DG_EINVAL, "NULL argument");
  switch (key) {
    case DG_OPT_EXCHANGE: *value = c->exchange; return DG_OK;
    case DG_OPT_XCD_REMAP: *value = c->xcd_remap; return DG_OK;
    case DG_OPT_ORDER: *value = c->order; return DG_OK;
    case DG_OPT_PENCIL_X: *value = c->pencil_x; return DG_OK;
    case DG_OPT_PENCIL_Z: *value = c->pencil_z; return DG_OK;
    case DG_OPT_VISC_FUSED: *value = c->visc_fused; return DG_OK;
    default: return fail(DG_EINVAL, "unknown option %d", key);
  }
}

size_t dg_workspace_bytes(const dg_ctx* c) {
  if (!c) return 0;
  return dg_workspace_layout(c).total;
}

int dg_set_workspace(dg_ctx* c, void* dptr, size_t bytes) {
  if (!c) return fail(DG_EINVAL, "NULL context");
  if (!dptr) return fail(DG_EINVAL, "NULL workspace");
  if (((uintptr_t)dptr) & 255) return fail(DG_EINVAL, "workspace not 256-byte aligned");
  const size_t need = dg_workspace_layout(c).total;
  if (bytes < need) return fail(DG_EWORKSPACE, "workspace %zu bytes < %zu", bytes, need);
  c->ws = (char*)dptr;
  c->ws_bytes = bytes;
  ++c->epoch;
  return DG_OK;
}

int64_t dg_num_dof(const dg_ctx* c) {
  if (!c) return -1;
  return c->E * c->N * c->N * c->N;
}

int dg_quadrature(int p, double* xi, double* w) {
  if (p < 0 || p >= DG_MAXN) return fail(DG_EUNSUPPORTED, "p must be in 0..%d", DG_MAXN - 1);
  if (!xi || !w) return fail(DG_EINVAL, "NULL output");
  gauss_legendre(p + 1, xi, w);
  return DG_OK;
}

int dg_rhs(dg_ctx* c, const double* Q, double* R) {
  int rc = check_ready(c);
  if (rc) return rc;
  rc = check_state_pair(c, Q, "Q", R, "R");
  if (rc) return rc;
  const bool f32 = c->precision == DG_FP32_MFMA;
  if (c->mu > 0.0 || c->volume_form == DG_VOLUME_KEP) {
    const bool fused = c->mu > 0.0 && visc_fused(c);
    int err = 0;
    if (!fused) {
      err = timed(c, TK_RHS, [&] { return euler_rate_nb(c, Q, R); });
      if (err) return hip_fail(err, "rhs launch");
    }
    if (c->mu == 0.0) return DG_OK;
    double* Fv = (double*)(c->ws + dg_workspace_layout(c).off_visc_fv);
    err = timed(c, TK_VISC,
                [&] { return dg_launch_visc(c, Q, Fv, R, nullptr, nullptr, 0, 0.0, 0.0, 0.0, 0, fused); });
    if (err) return hip_fail(err, "viscous rate launch");
    return DG_OK;
  }
  if (c->exchange == DG_EXCHANGE_NEIGHBOUR) {
    int err = timed(c, TK_RHS, [&] {
      return f32 ? dg_launch_stage_nb_f32(c, Q, nullptr, R, 0, 0.0, 0.0, 0.0, 0)
                 : dg_launch_stage_nb(c, Q, nullptr, R, 0, 0.0, 0.0, 0.0, 0);
    });
    if (err) return hip_fail(err, "rhs launch");
    return DG_OK;
  }
  int err = timed(c, TK_TRACE, [&] {
    return f32 ? dg_launch_trace_f32(c, Q, (char*)trace_buf(c, 0)) : dg_launch_trace(c, Q, trace_buf(c, 0));
  });
  if (err) return hip_fail(err, "trace launch");
  err = timed(c, TK_RHS, [&] {
    return f32 ? dg_launch_rhs_f32(c, Q, (const char*)trace_buf(c, 0), R) : dg_launch_rhs(c, Q, trace_buf(c, 0), R);
  });
  if (err) return hip_fail(err, "rhs launch");
  return DG_OK;
}

int dg_rk_stage(dg_ctx* c, int s, double* Q, double* res, double dt) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (s < 0 || s > 4) return fail(DG_EINVAL, "stage must be 0..4 (got %d)", s);
  if (!std::isfinite(dt)) return fail(DG_EINVAL, "dt must be finite");
  rc = check_state_pair(c, Q, "Q", res, "res");
  if (rc) return rc;
  return stages(c, Q, res, dt, s, 1);
}

int dg_rk_steps(dg_ctx* c, double* Q, double* res, double dt, int nsteps) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(dt)) return fail(DG_EINVAL, "dt must be finite");
  rc = check_state_pair(c, Q, "Q", res, "res");
  if (rc) return rc;
  if (nsteps == 0) return DG_OK;
  if ((int64_t)nsteps * 5 > 0x7fffffffLL) return fail(DG_EINVAL, "too many steps");
  return stages(c, Q, res, dt, 0, 5 * nsteps);
}

int dg_rk_step(dg_ctx* c, double* Q, double* res, double dt) { return dg_rk_steps(c, Q, res, dt, 1); }

int dg_rk_steps_noalloc(dg_ctx* c, double* Q, double* res, double dt, int nsteps) {
  if (!c) return fail(DG_EINVAL, "NULL context");
  if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(dt)) return fail(DG_EINVAL, "dt must be finite");
  int rc = check_state_pair(c, Q, "Q", res, "res");
  if (rc) return rc;
  if (c->mu > 0.0) return fail(DG_EUNSUPPORTED, "dg_rk_steps_noalloc covers the Euler terms only (viscosity is set)");
  if (c->volume_form == DG_VOLUME_KEP)
    return fail(DG_EUNSUPPORTED, "dg_rk_steps_noalloc covers the standard volume form only (the split form is set)");
  if (state_bytes(c) > kScratchBytes)
    return fail(DG_EUNSUPPORTED, "state of %zu bytes exceeds the %zu-byte static buffer of dg_rk_steps_noalloc",
                state_bytes(c), kScratchBytes);
  if (nsteps == 0) return DG_OK;
  if ((int64_t)nsteps * 5 > 0x7fffffffLL) return fail(DG_EINVAL, "too many steps");
  double* q2 = nullptr;
  rc = scratch_of_current_device(&q2);
  if (rc) return rc;
  return stages_nb(c, Q, res, dt, 0, 5 * nsteps, q2, false);
}

int dg_rk_graph_steps(dg_ctx* c, double* Q, double* res, double dt, int nsteps) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(dt)) return fail(DG_EINVAL, "dt must be finite");
  rc = check_state_pair(c, Q, "Q", res, "res");
  if (rc) return rc;
  if (nsteps == 0) return DG_OK;
  if (c->exchange != DG_EXCHANGE_NEIGHBOUR || c->mu > 0.0 || c->volume_form == DG_VOLUME_KEP)
    return stages(c, Q, res, dt, 0, 5 * nsteps);
  int err;
  if (!c->gstream) {
    err = (int)hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking);
    if (err) return hip_fail(err, "graph stream");
    err = (int)hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming);
    if (err) return hip_fail(err, "graph event");
    err = (int)hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming);
    if (err) return hip_fail(err, "graph event");
  }
  if (c->gQ != Q || c->gR != res || c->gdt != dt || c->gepoch != c->epoch) {
    for (int k = 0; k < 2; ++k) {
      if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
      c->gexec[k] = nullptr;
    }
  }
  // the graph stream runs after the caller's stream, and the caller's
  // stream after it
  err = (int)hipEventRecord(c->ev_in, c->stream);
  if (err) return hip_fail(err, "event record");
  err = (int)hipStreamWaitEvent(c->gstream, c->ev_in, 0);
  if (err) return hip_fail(err, "stream wait");
  double* buf[2] = {Q, q2_buf(c)};
  for (int par = 0; par < 2; ++par) {
    if (c->gexec[par]) continue;
    // one step = five stage launches; a step that starts from buf[par]
    // (stage count before it of parity par) alternates from there
    hipGraph_t graph = nullptr;
    const hipStream_t user = c->stream;
    c->stream = c->gstream;
    err = (int)hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal);
    int lerr = 0;
    for (int s = 0; s < 5 && !err && !lerr; ++s) {
      const int g = par + s;
      lerr = c->precision == DG_FP32_MFMA
                 ? dg_launch_stage_nb_f32(c, buf[g & 1], buf[(g + 1) & 1], res, 1, kRKA[s], kRKB[s], dt, s == 0)
                 : dg_launch_stage_nb(c, buf[g & 1], buf[(g + 1) & 1], res, 1, kRKA[s], kRKB[s], dt, s == 0);
    }
    const int cerr = err ? err : (int)hipStreamEndCapture(c->gstream, &graph);
    c->stream = user;
    if (err) return hip_fail(err, "begin capture");
    if (lerr || cerr) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(lerr ? lerr : cerr, "capture");
    }
    err = (int)hipGraphInstantiate(&c->gexec[par], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (err) return hip_fail(err, "graph instantiate");
  }
  c->gQ = Q;
  c->gR = res;
  c->gdt = dt;
  c->gepoch = c->epoch;
  for (int n = 0; n < nsteps; ++n) {
    err = (int)hipGraphLaunch(c->gexec[n & 1], c->gstream);
    if (err) return hip_fail(err, "graph launch");
  }
  if (nsteps & 1) {
    err = (int)hipMemcpyAsync(Q, buf[1], state_bytes(c), hipMemcpyDeviceToDevice, c->gstream);
    if (err) return hip_fail(err, "state copy");
  }
  err = (int)hipEventRecord(c->ev_out, c->gstream);
  if (err) return hip_fail(err, "event record");
  err = (int)hipStreamWaitEvent(c->stream, c->ev_out, 0);
  if (err) return hip_fail(err, "stream wait");
  return DG_OK;
}

int dg_rhs_vjp(dg_ctx* c, const double* Q, const double* gR, double* gQ) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (c->mu > 0.0) return fail(DG_EUNSUPPORTED, "the adjoint covers the Euler terms only (viscosity is set)");
  if (c->volume_form == DG_VOLUME_KEP)
    return fail(DG_EUNSUPPORTED, "the adjoint covers the standard volume form only (the split form is set)");
  if (!Q || !gR || !gQ) return fail(DG_EINVAL, "NULL array");
  if (misaligned(Q) || misaligned(gR) || misaligned(gQ)) return fail(DG_EINVAL, "arrays must be 8-byte aligned");
  if (overlap(Q, gQ, state_bytes(c))) return fail(DG_EALIAS, "gQ overlaps Q");
  if (overlap(gR, gQ, state_bytes(c))) return fail(DG_EALIAS, "gQ overlaps gR");
  int err = timed(c, TK_VJP, [&] { return dg_launch_vjp(c, Q, gR, gQ, c->ws); });
  if (err) return hip_fail(err, "vjp launch");
  return DG_OK;
}

int dg_rk_stage_vjp(dg_ctx* c, int s, const double* Qs, double* gQ, double* gres, double dt) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (c->mu > 0.0) return fail(DG_EUNSUPPORTED, "the adjoint covers the Euler terms only (viscosity is set)");
  if (c->volume_form == DG_VOLUME_KEP)
    return fail(DG_EUNSUPPORTED, "the adjoint covers the standard volume form only (the split form is set)");
  if (s < 0 || s > 4) return fail(DG_EINVAL, "stage must be 0..4 (got %d)", s);
  if (!std::isfinite(dt)) return fail(DG_EINVAL, "dt must be finite");
  if (!Qs || !gQ || !gres) return fail(DG_EINVAL, "NULL array");
  if (misaligned(Qs) || misaligned(gQ) || misaligned(gres)) return fail(DG_EINVAL, "arrays must be 8-byte aligned");
  const size_t sb = state_bytes(c);
  if (overlap(gQ, gres, sb)) return fail(DG_EALIAS, "gQ overlaps gres");
  if (overlap(Qs, gQ, sb) || overlap(Qs, gres, sb)) return fail(DG_EALIAS, "adjoint overlaps Qs");
  const DGWorkspace L = dg_workspace_layout(c);
  double* gtot = (double*)(c->ws + L.off_vjp);
  double* v = (double*)(c->ws + L.off_vjp + align256(sb));
  const int64_t n = (int64_t)(sb / sizeof(double));
  int err = timed(c, TK_VJP, [&] { return dg_launch_axpy(c, n, gres, kRKB[s], gQ, gtot); });
  if (err) return hip_fail(err, "axpy launch");
  err = timed(c, TK_VJP, [&] { return dg_launch_vjp(c, Qs, gtot, v, c->ws); });
  if (err) return hip_fail(err, "vjp launch");
  err = timed(c, TK_VJP, [&] { return dg_launch_rk_reverse(c, n, v, dt, kRKA[s], gtot, gQ, gres); });
  if (err) return hip_fail(err, "reverse stage launch");
  return DG_OK;
}

int dg_kinetic_energy_grad(dg_ctx* c, const double* Q, double* gQ) {
  int rc = check_ready(c);
  if (rc) return rc;
  rc = check_state_pair(c, Q, "Q", gQ, "gQ");
  if (rc) return rc;
  int err = timed(c, TK_VJP, [&] { return dg_launch_ke_grad(c, Q, gQ); });
  if (err) return hip_fail(err, "kinetic-energy gradient launch");
  return DG_OK;
}

int dg_recip_sqrt(const double* x, double* r, double* s, int64_t n, void* stream) {
  if (n < 0) return fail(DG_EINVAL, "n must be >= 0");
  if (n == 0) return DG_OK;
  if (!x || !r || !s) return fail(DG_EINVAL, "NULL array");
  if (misaligned(x) || misaligned(r) || misaligned(s)) return fail(DG_EINVAL, "arrays must be 8-byte aligned");
  const size_t b = (size_t)n * sizeof(double);
  if (overlap(x, r, b) || overlap(x, s, b) || overlap(r, s, b)) return fail(DG_EALIAS, "arrays overlap");
  int err = dg_launch_recip_root((hipStream_t)stream, x, r, s, n);
  if (err) return hip_fail(err, "recip/sqrt launch");
  return DG_OK;
}

int dg_integrals(dg_ctx* c, const double* Q, double out[6]) {
  if (!out) return fail(DG_EINVAL, "NULL output");
  double v[DG_RED_VALS];
  int rc = run_reduce(c, Q, v);
  if (rc) return rc;
  for (int i = 0; i < 6; ++i) out[i] = v[i];
  return DG_OK;
}

int dg_max_wavespeed(dg_ctx* c, const double* Q, double* out) {
  if (!out) return fail(DG_EINVAL, "NULL output");
  double v[DG_RED_VALS];
  int rc = run_reduce(c, Q, v);
  if (rc) return rc;
  *out = v[6];
  return DG_OK;
}

int dg_check_state(dg_ctx* c, const double* Q) {
  double v[DG_RED_VALS];
  int rc = run_reduce(c, Q, v);
  if (rc) return rc;
  if (v[7] > 0) return fail(DG_ENONPHYSICAL, "%.0f node(s) with rho<=0, p<=0 or non-finite values", v[7]);
  return DG_OK;
}

}  // extern "C"
